/*
 * qpm.h -- C ABI of the MI355X (gfx950) hot path of HWSDA, the hybrid
 * differential-evolution / grey-wolf optimiser for aperiodically poled
 * quasi-phase-matching crystals (He Chen, Zihua Zheng, Jinghua Sun, "Design
 * of quasi phase matching crystal based on differential gray wolf
 * algorithm").
 *
 * Objective (paper Sec. 2.1, the d_eff double integral): for a crystal cut
 * into N domains [z_{n-1}, z_n) with polarity d_n = +1 or -1,
 *   d_eff = int d(z) e^{-i dk2 z} ( int_{z_0}^{z} d(x) e^{-i dk1 x} dx ) dz,
 * and the fitness is f = |d_eff|^2 (maximised; the undepleted-pump
 * prefactor is dropped, as in the paper). Units: z in um, dk in 1/um,
 * d_eff in um^2, f in um^4.
 *
 * Conventions shared by every entry point
 *   - Device pointers are HIP device memory of the current device; host
 *     pointers are ordinary process memory. The caller owns every buffer it
 *     passes and the library keeps no caller pointer after a call returns.
 *   - qpm_stream is a hipStream_t (NULL = the null stream). Entry points
 *     validate their arguments on the host, enqueue work on the stream and
 *     return without synchronising unless stated otherwise; device faults
 *     surface at the next synchronisation.
 *   - A failing call returns a negative qpm_status, launches nothing and
 *     writes no output; qpm_last_error() then holds a message (per thread).
 *     Nothing aborts and no C++ exception crosses the ABI.
 *   - Bit layout of a population of +-1 sequences ("population-major"):
 *     uint32 words bits[w * ld + i], w < W = ceil(N / 32), i < ld; bit k of
 *     word w of genome i is set exactly when d_{32 w + k} = -1 (0-based
 *     domains). ld >= np and ld is a multiple of 64. Padding bits (domains
 *     >= N) must be 0; padding columns (i >= np) are read but ignored.
 *   - Genes (the optimiser's continuous positions): float rows x[i * ldx + j],
 *     j < D = N, ldx >= D rounded up to a multiple of 4, rows 16-byte
 *     aligned. Gene j maps to d_j = -1 exactly when x_ij < 0.0f (so -0.0
 *     maps to +1).
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the
 *     64-bit seed; the counter is (c0, individual, generation,
 *     instance << 8 | stream tag), so every draw depends only on its
 *     coordinates, never on launch shape.
 *   - Scratch: the evaluation entry points on a design or an objective
 *     (fitness, objective, relaxation) keep their device scratch with that
 *     handle between calls, one buffer per stream handle for up to 4
 *     streams, freed with the handle. Successive
 *     uses of a buffer are ordered by its stream, and one host lock per
 *     handle covers a call's enqueueing, so calls from several streams and
 *     threads are safe. Calls under stream capture, or on a fifth stream,
 *     take scratch from the stream-ordered allocator of s instead.
 */
#ifndef QPM_H
#define QPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qpm_status;
enum {
    QPM_OK = 0,
    QPM_EINVAL = -1,  /* an argument is invalid (see each entry point) */
    QPM_ERANGE = -2,  /* a size overflows the supported range */
    QPM_ENOMEM = -3,  /* a device allocation failed */
    QPM_EHIP = -4,    /* a HIP runtime call failed (text in qpm_last_error) */
    QPM_ENOTSUP = -5  /* the current device is not gfx950 */
};

typedef enum {
    QPM_PREC_F32 = 0, /* FP32 within blocks of domains, FP64 across blocks */
    QPM_PREC_F64 = 1  /* FP64 throughout */
} qpm_prec;

/* Which fitness kernel evaluates a population. */
typedef enum {
    QPM_FIT_AUTO = 0,       /* the table kernel, launch shape from the tuner in runs */
    QPM_FIT_SEGMENTED = 1,  /* domain axis split over waves and workgroups, per-domain walk */
    QPM_FIT_PER_GENOME = 2, /* one lane per genome over all N (FP64 only) */
    QPM_FIT_TABLE = 3       /* segmented, each 4-domain block's triple looked up
                               by its sign pattern in a per-design table (LDS) */
} qpm_fit_kernel;

typedef void *qpm_stream;               /* a hipStream_t */
typedef struct qpm_design_s *qpm_design; /* owns the device phase tables */
typedef struct qpm_run_s *qpm_run_handle;
typedef struct qpm_batch_s *qpm_batch;   /* many designs, concatenated tables */
typedef struct qpm_batch_run_s *qpm_batch_run_handle;
typedef struct qpm_objective_s *qpm_objective; /* K designs, one objective */

/* Status text for a code, and the calling thread's last error message. */
const char *qpm_status_string(qpm_status s);
const char *qpm_last_error(void);

/*
 * qpm_precompute_phases -- build a design: the per-domain integrals of the
 * d_eff double integral (paper Sec. 2.1), evaluated on the GPU in FP64.
 *   a_n = int_{z_{n-1}}^{z_n} e^{-i dk1 x} dx,
 *   b_n = int_{z_{n-1}}^{z_n} e^{-i dk2 z} dz,
 *   c_n = int_{z_{n-1}}^{z_n} e^{-i dk2 z} int_{z_{n-1}}^{z} e^{-i dk1 x} dx dz,
 *   C = sum_n c_n, so that d_eff = sum_n d_n b_n P_{n-1} + C with
 *   P_n = sum_{m<=n} d_m a_m.
 * z: host, n_domains + 1 finite, strictly increasing boundaries (um); z[0]
 * may be non-zero. dk1, dk2: finite (1/um), zero allowed. n_domains >= 1
 * and <= 2^27. The call synchronises s before it returns (the design is
 * ready to use on any stream). *out receives the design; free it with
 * qpm_design_free. Errors: QPM_EINVAL (bad z or dk, NULL pointer),
 * QPM_ERANGE (n too large), QPM_ENOMEM, QPM_EHIP, QPM_ENOTSUP.
 */
qpm_status qpm_precompute_phases(const double *z, int64_t n_domains, double dk1, double dk2,
                                 qpm_stream s, qpm_design *out);

/* Release a design (NULL is accepted). Synchronises the device first. */
qpm_status qpm_design_free(qpm_design d);

/* n_domains and C = sum_n c_n (re, im) of a design (host outputs; either
 * may be NULL). */
qpm_status qpm_design_info(qpm_design d, int64_t *n_domains, double *C);

/* Copy the FP64 per-domain integrals to host arrays of 2 * n_domains
 * doubles (re, im interleaved); any pointer may be NULL. Synchronous. */
qpm_status qpm_design_read_phases(qpm_design d, double *a, double *b, double *c);

/*
 * qpm_eval_fitness -- f_i = |d_eff(d_i)|^2 for np genomes (paper Sec. 2.1;
 * evaluation step of Sec. 3.2).
 * bits: device, population-major words (layout above), W x ld uint32.
 * fitness: device, np floats (QPM_PREC_F32) or doubles (QPM_PREC_F64).
 * kernel: a qpm_fit_kernel; QPM_FIT_PER_GENOME needs QPM_PREC_F64.
 * Device scratch: the segment partials (see Conventions, Scratch).
 * Errors: QPM_EINVAL (np < 1, ld < np or not a multiple of 64, NULL
 * pointer, unknown precision or kernel), QPM_ENOMEM, QPM_EHIP.
 */
qpm_status qpm_eval_fitness(qpm_design d, qpm_prec p, const uint32_t *bits, int64_t np,
                            int64_t ld, void *fitness, int32_t kernel, qpm_stream s);

/*
 * qpm_eval_fitness_noalloc -- qpm_eval_fitness for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): same arguments, launch plan and
 * results (bit for bit), but the segment partials live in a fixed 16 MiB
 * device array of the library, one per device, held until the process
 * ends; the call allocates and frees nothing. Every call on a device shares
 * that device's array, so calls that overlap on one device (other streams,
 * other threads) race; the caller orders them. Errors: as qpm_eval_fitness,
 * and QPM_ERANGE when the population needs more than 16 MiB of partials
 * (6 doubles per genome column ld and workgroup segment; the 4096 x 10^4
 * fitness workload needs 3.1 MB).
 */
qpm_status qpm_eval_fitness_noalloc(qpm_design d, qpm_prec p, const uint32_t *bits, int64_t np,
                                    int64_t ld, void *fitness, int32_t kernel, qpm_stream s);

/*
 * qpm_eval_fitness_shape -- qpm_eval_fitness with the segmented kernel's
 * launch shape given explicitly (for tuning): waves_per_group in
 * {1, 2, 4, 8, 16} waves of 64 genomes share one workgroup and scan
 * consecutive segments of words_per_wave >= 1 bit words each. The result
 * equals qpm_eval_fitness up to the summation order of the segments.
 */
qpm_status qpm_eval_fitness_shape(qpm_design d, qpm_prec p, const uint32_t *bits, int64_t np,
                                  int64_t ld, void *fitness, int32_t waves_per_group,
                                  int32_t words_per_wave, qpm_stream s);

/*
 * qpm_eval_fitness_table_shape -- qpm_eval_fitness with the table kernel
 * (QPM_FIT_TABLE) and its launch shape given explicitly: a workgroup holds
 * groups_per_workgroup in {1, 2, 4} groups of 64 genomes x 4 waves, each
 * wave scanning words_per_wave >= 1 bit words; the tables of the
 * workgroup's 4 words_per_wave words are staged in LDS (3 KB per word in
 * FP32, 6 KB in FP64), which must fit in 64 KB. The result equals
 * qpm_eval_fitness with QPM_FIT_TABLE up to the summation order.
 * Errors: as qpm_eval_fitness, QPM_EINVAL for a shape outside these limits.
 */
qpm_status qpm_eval_fitness_table_shape(qpm_design d, qpm_prec p, const uint32_t *bits, int64_t np,
                                        int64_t ld, void *fitness, int32_t groups_per_workgroup,
                                        int32_t words_per_wave, qpm_stream s);

/*
 * qpm_init_population -- DE step 1 (paper Sec. 2.2.1): x_ij uniform on
 * [-1, 1) (Philox stream INIT, counter (j / 4, i, 0, inst << 8 | 1), word
 * j % 4, value (u >> 8) 2^-23 - 1), and the +-1 bits of every row.
 * x: device np x ldx floats; bits: device W x ld words.
 */
qpm_status qpm_init_population(int64_t np, int64_t D, int64_t ldx, uint64_t seed, uint32_t inst,
                               float *x, uint32_t *bits, int64_t ld, qpm_stream s);

/*
 * qpm_de_step -- DE rand/1 mutation and binomial crossover (paper Sec.
 * 2.2.1 steps 2-3), synchronous over the population x of generation g:
 *   r1, r2, r3 distinct and != i (np >= 4), drawn without replacement from
 *   one Philox call (counter (0, i, g, inst << 8 | 2): words 0..2 give
 *   k_m = floor(u np_m / 2^32) with np_m = np-1, np-2, np-3 and r_m the k_m-th
 *   index not yet excluded; word 3 gives jrand = floor(u D / 2^32));
 *   v_j = fmaf(F, x_r2j - x_r3j, x_r1j) clamped to [-1, 1];
 *   u_ij = v_j if ((u >> 8) 2^-24 <= CR) or j == jrand, else x_ij, with u
 *   from counter (j / 4, i, g, inst << 8 | 3), word j % 4.
 * x: device np x ldx; u: device np x ldx (trial vectors); u_bits: device
 * W x ld words of the trials. F in [0, 2], CR in [0, 1].
 * Errors: QPM_EINVAL (np < 4, D < 1, ldx, ld, F, CR out of range, NULL or
 * misaligned pointer).
 */
qpm_status qpm_de_step(const float *x, int64_t np, int64_t D, int64_t ldx, float F, float CR,
                       uint64_t seed, uint32_t generation, uint32_t inst, float *u,
                       uint32_t *u_bits, int64_t ld, qpm_stream s);
/*
 * qpm_de_step_shape -- qpm_de_step with an explicit launch shape: each wave
 * covers individuals_per_wave individuals (1, 2 or 4; 0 = chosen from np)
 * of a gene chunk of 256 / individuals_per_wave genes, and each workgroup
 * makes `passes` (1, 2 or 4) passes over consecutive groups of
 * individuals. The shape changes the speed only, never the result.
 * Errors: as qpm_de_step, and QPM_EINVAL for a shape outside these sets.
 */
qpm_status qpm_de_step_shape(const float *x, int64_t np, int64_t D, int64_t ldx, float F, float CR,
                             uint64_t seed, uint32_t generation, uint32_t inst, float *u,
                             uint32_t *u_bits, int64_t ld, int32_t individuals_per_wave,
                             int32_t passes, qpm_stream s);

/*
 * qpm_gwo_step -- grey-wolf update of the omega wolves (paper Sec. 2.2.2):
 * per gene j of a non-leader i and leader k in (alpha, beta, delta), with
 * r1 = lo16(u) 2^-16 and r2 = hi16(u) 2^-16 of one Philox word,
 *   A = fmaf(2a, r1, -a), C = 2 r2, D_k = |fmaf(C, X_kj, -x_ij)|,
 *   Y_k = fmaf(-A, D_k, X_kj);
 * variant 0 (as printed): y = (sum_k |Y_k| Y_k / sum_k |Y_k|) / 3 (0 if the
 * sum is 0); variant 1: y = (Y_1 + Y_2 + Y_3) / 3; clamped to [-1, 1].
 * Philox words: for gene quad q = j / 4 and t = 3 (j % 4) + k, counter
 * (3 q + t / 4, i, g, inst << 8 | 4), word t % 4.
 * leaders: host int32[3] (alpha, beta, delta), distinct, in [0, np),
 * validated before the launch and passed by value (the call enqueues on s
 * and returns without synchronising). Leader rows of y and y_bits are left
 * untouched. a = 0 or
 * 2^-100 <= a <= 1e30 (the parameter runs from 2 down to 0).
 */
/*
 * qpm_dgwo_step -- the improved discrete four-leader grey-wolf step of paper
 * Sec. 3.1.2. The paper describes it in words only (four leaders, +-1
 * states, a transition probability from the leaders' state counts, strong
 * perturbation early and a small flip probability late, social learning
 * at a falling rate); this is the library's reading of it, with no rate
 * taken from the paper. For gene j of a non-leader i, with one Philox word
 * w (counter (j / 4, i, g, inst << 8 | 5), word j % 4) and
 * params = {t, 1 - 2 eps, eps, lambda} (a run uses t = g / G,
 * eps = 0.1 (1 - t) + 0.01 t, lambda = 0.2 (1 - t), each rounded to float):
 *   n = number of the 4 leaders with gene >= 0 at j; dist = n / 4;
 *   maj = 1, 0 or 1/2 for n > 2, n < 2, n = 2;
 *   p = fmaf(t, maj - dist, dist); p' = fmaf(1 - 2 eps, p, eps);
 *   y = the state of leader w >> 30 when (w >> 16 & 0x3FFF) 2^-14 < lambda
 *   (social learning), else +1 when (w & 0xFFFF) 2^-16 < p', else -1.
 * leaders: host int32[4], distinct, in [0, np): alpha, beta, delta (their
 * rows of y and y_bits are left untouched) and the fourth; validated before
 * the launch and passed by value (no synchronisation). params: host.
 * Errors: as qpm_gwo_step, and QPM_EINVAL for non-finite params.
 */
qpm_status qpm_dgwo_step(const float *x, int64_t np, int64_t D, int64_t ldx, const int32_t *leaders,
                         const float *params, uint64_t seed, uint32_t generation, uint32_t inst, float *y,
                         uint32_t *y_bits, int64_t ld, qpm_stream s);

qpm_status qpm_gwo_step(const float *x, int64_t np, int64_t D, int64_t ldx,
                        const int32_t *leaders, float a, uint64_t seed, uint32_t generation,
                        uint32_t inst, int32_t variant, float *y, uint32_t *y_bits, int64_t ld,
                        qpm_stream s);

/*
 * qpm_relax_forward -- the relaxation d = tanh(theta) of a design (not in
 * the paper; it extends the d_eff double integral of Sec. 2.1 to real d):
 *   S = sum_{m<n} d_m d_n a_m b_n + sum_n d_n^2 c_n,  f = |S|^2,
 * which equals the +-1 fitness where |theta| is large. theta: device,
 * B x ldt floats (row b holds theta_{b,0..N-1}); f: device B floats and/or
 * S: device B x 2 doubles (re, im); either may be NULL, not both.
 * edges: NULL, or device doubles (qpm_relax_edges_size of them) that
 * receive the per-segment prefix and suffix sums the adjoint needs, so that
 * qpm_relax_backward given them skips recomputing the forward pass.
 * prec selects how tanh is evaluated: FP32 (binary32, hardware exp2 and
 * reciprocal) or FP64; the sums are FP64 in both (for FP32 the
 * sub-segment sums kept in edges are stored rounded to binary32). Device
 * scratch: the segment partials (see Conventions, Scratch).
 * Errors: QPM_EINVAL (NULL design or theta, both outputs NULL, B outside
 * [1, 2^24], ldt < N, unknown precision), QPM_ERANGE, QPM_EHIP.
 */
qpm_status qpm_relax_forward(qpm_design d, qpm_prec p, const float *theta, int64_t B, int64_t ldt,
                             float *f, double *S, double *edges, qpm_stream s);

/* Number of doubles of the edges buffer of qpm_relax_forward for a batch of
 * B rows in precision p: per row, 4 doubles per segment of 128 domains (the
 * prefix A before the segment and the sum of B from it on) and 4 values per
 * sub-segment of 32 domains (its own sums A and B: doubles for QPM_PREC_F64,
 * floats, 2 doubles' worth, for QPM_PREC_F32). */
qpm_status qpm_relax_edges_size(qpm_design d, qpm_prec p, int64_t B, int64_t *count);

/*
 * qpm_relax_backward -- the adjoint of qpm_relax_forward:
 *   grad_theta_{b,k} = grad_f_b 2 Re(conj(S_b) dS_b/dd_k) (1 - d_k^2),
 *   dS/dd_k = b_k P_{k-1} + a_k R_{k+1} + 2 c_k d_k,
 * with P_{k-1} = sum_{m<k} d_m a_m and R_{k+1} = sum_{n>k} d_n b_n.
 * S: device B x 2 doubles saved from the forward call; edges: the edges of
 * the same forward call (same theta and precision), or NULL to recompute
 * them; grad_f: device B floats; grad_theta: device B x ldg floats (entries
 * past N are not written).
 * Errors: as qpm_relax_forward, and QPM_EINVAL for NULL S, grad_f or
 * grad_theta or ldg < N.
 */
qpm_status qpm_relax_backward(qpm_design d, qpm_prec p, const float *theta, int64_t B, int64_t ldt,
                              const double *S, const double *edges, const float *grad_f,
                              float *grad_theta, int64_t ldg, qpm_stream s);

/*
 * Multi-wavelength objective (the paper's multi-wavelength second- and
 * coupled third-harmonic designs, its last section). K designs made by
 * qpm_precompute_phases from the same boundaries z, one per wavelength
 * (its dk1, dk2); L = z_N - z_0. Per genome and design k:
 *   QPM_OBJ_SHG  G_k = |sum_n d_n a_n| / L, the single-integral coupling of
 *                second-harmonic generation with the design's dk1 (dk2 is
 *                not used);
 *   QPM_OBJ_THG  G_k = |d_eff,k| / L^2, the coupled double integral of
 *                Sec. 2.1 with the design's (dk1, dk2).
 * The paper minimises h = sum_k |G0 - G_k| + beta (max_k G_k - min_k G_k);
 * fitness = -h is maximised. G is normalised (at most 1) so that G0 and
 * beta are dimensionless (a reading: the paper does not give its scale).
 * One bit stream serves all K designs: each bit word is loaded once and
 * looked up in the K designs' sign-pattern tables.
 */
typedef enum { QPM_OBJ_SHG = 0, QPM_OBJ_THG = 1 } qpm_objective_kind;

/* designs: host array of K (1..8) designs that share their boundaries
 * (checked: N, z_0, z_N and a hash of z), on the current device; the
 * objective refers to them, so they must outlive it (and any run on it).
 * G0, beta: finite. Errors: QPM_EINVAL (NULL, K out of range, unknown
 * kind, boundaries differ, non-finite G0 or beta). */
qpm_status qpm_objective_create(const qpm_design *designs, int32_t K, int32_t kind, double G0, double beta,
                                qpm_objective *out);
qpm_status qpm_objective_free(qpm_objective o); /* NULL accepted */

/* fitness = -h per genome (device, np floats for QPM_PREC_F32 or doubles
 * for QPM_PREC_F64) and, when G is not NULL, G_k of genome i at
 * G[k * ldG + i] (device doubles, ldG >= np). bits: as qpm_eval_fitness.
 * Errors: as qpm_eval_fitness, and QPM_EINVAL for ldG < np. */
qpm_status qpm_eval_objective(qpm_objective o, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                              void *fitness, double *G, int64_t ldG, qpm_stream s);

/* qpm_eval_objective with an explicit launch shape: a workgroup is 64
 * genomes x 4 segment waves of words_per_wave bit words each, in [1, 5]
 * (FP32) or [1, 2] (FP64); the default picks it from N and np. Results
 * equal qpm_eval_objective's up to the summation order. Errors: as
 * qpm_eval_objective, QPM_EINVAL for words_per_wave out of range,
 * QPM_ERANGE when the words need more than 65535 workgroup segments. */
qpm_status qpm_eval_objective_shape(qpm_objective o, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                    void *fitness, double *G, int64_t ldG, int32_t words_per_wave,
                                    qpm_stream s);

/* Configuration of a whole optimisation (paper Sec. 3.2, steps 1-7). */
typedef struct {
    int64_t np;          /* population size, >= 4 */
    int64_t generations; /* G >= 1 */
    float F;             /* DE scale factor in [0, 2] */
    float CR;            /* crossover rate in [0, 1] */
    uint64_t seed;       /* Philox key */
    uint32_t inst;       /* instance number in the Philox counter */
    int32_t prec;        /* qpm_prec of the fitness kernel */
    int32_t gwo_variant; /* 0 = weighted as printed, 1 = plain mean,
                            2 = discrete four-leader step (qpm_dgwo_step;
                            a_g unused; the fourth leader is the best
                            genome after alpha, beta, delta) */
    int32_t use_graph;   /* 1 = replay one captured generation */
    int32_t fit_kernel;  /* qpm_fit_kernel of the evaluations */
    int32_t tune;        /* 1 = time candidate launch shapes of the fitness
                            and DE kernels at creation and keep the fastest
                            (cached per problem size; QPM_TUNE_CACHE file) */
    int32_t control;     /* qpm_control: how F_g and a_g are set */
    int32_t trials;      /* qpm_trials: where the DE trial genes go */
    int32_t algo;        /* qpm_algo: HWSDA, or one of its two parts alone */
    int32_t fused;       /* whole generations in one workgroup with the
                            population in LDS: 0 = when the run allows it
                            (table or automatic kernel, fixed or decaying
                            control, gwo_variant 0 or 1, no objective,
                            np <= 64 and the population within 160 KB of
                            LDS), 1 = required (QPM_ENOTSUP otherwise),
                            -1 = never. FP64: the same trajectory as the
                            multi-kernel path. FP32: the fitness is walked
                            with the FP64 tables and rounded to binary32 (at
                            least the FP32 path's accuracy), so a near tie
                            may be decided otherwise than there */
} qpm_run_config;

/*
 * The optimiser a run applies each generation. HWSDA is the hybrid of paper
 * Sec. 3.2; the other two are the optimisers it is compared with in the
 * tables of Sec. 4 (each alone, on the same fitness and random streams):
 *   QPM_ALGO_HWSDA  DE trials + greedy selection, leaders, grey-wolf
 *                   candidates + greedy selection (leaders kept);
 *   QPM_ALGO_DE     DE rand/1 alone (Sec. 2.2.1): trials, evaluation,
 *                   greedy selection; the leaders reported are the three
 *                   best after the selection;
 *   QPM_ALGO_GWO    the grey-wolf optimiser alone (Sec. 2.2.2): alpha,
 *                   beta, delta = the three best of the current population,
 *                   every other wolf moves to its candidate unconditionally
 *                   (the basic method has no greedy selection), evaluation;
 *                   gwo_variant applies as in HWSDA, F is unused.
 * DE and GWO runs store every trial (QPM_TRIALS_AUTO means STORE;
 * QPM_TRIALS_ACCEPTED is QPM_EINVAL). Batched runs take QPM_ALGO_HWSDA only.
 */
typedef enum { QPM_ALGO_HWSDA = 0, QPM_ALGO_DE = 1, QPM_ALGO_GWO = 2 } qpm_algo;

/*
 * Trial storage of a run's DE step (results are identical; speed differs):
 *   QPM_TRIALS_AUTO      ACCEPTED when the two gene buffers exceed 64 MB
 *                        and np <= 65536, else STORE;
 *   QPM_TRIALS_STORE     every trial's genes are written, selection keeps
 *                        or drops them;
 *   QPM_TRIALS_ACCEPTED  the DE step writes the trials' bits only; after
 *                        the selection, the accepted trials' genes are
 *                        computed again from the same draws and written
 *                        (np <= 65536, else QPM_EINVAL).
 */
typedef enum { QPM_TRIALS_AUTO = 0, QPM_TRIALS_STORE = 1, QPM_TRIALS_ACCEPTED = 2 } qpm_trials;
/* (Runs of batched designs take STORE for AUTO and accept ACCEPTED too.) */

/*
 * Parameter control (paper Sec. 3.1.1 and the parameter settings of
 * Sec. 4), with t = g / G evaluated in double and rounded to float once:
 *   QPM_CONTROL_FIXED     F_g = cfg->F, a_g = 2 (1 - t) (Sec. 2.2.2);
 *   QPM_CONTROL_DECAY     F_g = a_g = 0.1 (1 - t) + 0.01 t: F and a start at
 *                         0.1 and fall to 0.01 (the paper gives no decay
 *                         law; linear is this library's reading);
 *   QPM_CONTROL_ADAPTIVE  a_g as in DECAY; F_g in [0.01, 0.1] from the
 *                         fitness of the population entering generation g:
 *                         s = std f / mean f (population std),
 *                         kappa = (max f - mean f) / max f,
 *                         range = max f - min f (um^2); factor m = 1.2 if
 *                         s < 0.1 or kappa < 0.1 (low diversity: explore),
 *                         else 0.8 if s > 0.5 or range < 1e3 (exploit),
 *                         else 1; F_g = clamp(m base(g), 0.01, 0.1) with
 *                         base(g) = 0.1 (cos(pi t / 2) + 1) / 2 (1 - 0.2 t^2),
 *                         the cosine decay times the quadratic coefficient
 *                         from 1.0 to 0.8 (thresholds 0.5, factors, the
 *                         scale 0.1 and the definitions of s and kappa are
 *                         readings: the paper gives no values for them).
 * CR stays cfg->CR under every control. Runs of batched designs support
 * QPM_CONTROL_FIXED only (QPM_ENOTSUP otherwise).
 */
typedef enum { QPM_CONTROL_FIXED = 0, QPM_CONTROL_DECAY = 1, QPM_CONTROL_ADAPTIVE = 2 } qpm_control;

typedef struct {
    double best_fitness;  /* f of the best individual */
    int64_t best_index;   /* its slot (lowest slot among ties) */
    int64_t generations;  /* generations completed */
    int64_t fitness_evals; /* genomes evaluated */
    double domain_evals;  /* fitness_evals * N */
} qpm_run_stats;

/*
 * qpm_run_create -- allocate a run and perform step 1 (initialise, evaluate,
 * pick leaders). One generation g (steps 2-6 of paper Sec. 3.2) is then:
 * DE trials (qpm_de_step) with F_g, evaluation, greedy one-to-one
 * selection (a trial replaces its target only when strictly better),
 * leaders alpha, beta, delta = the three best by (f descending, slot
 * ascending), GWO candidates for every other wolf with a_g, evaluation,
 * greedy selection again (leaders excluded); F_g and a_g per cfg->control
 * (qpm_control). cfg->algo selects HWSDA or one of its parts alone
 * (qpm_algo). The run owns its own stream; s is the stream the caller's
 * later reads are ordered with. Errors: QPM_EINVAL for an out-of-range
 * field (np, G, F, CR, prec, gwo_variant, inst, fit_kernel, control,
 * trials, algo).
 */
qpm_status qpm_run_create(qpm_design d, const qpm_run_config *cfg, qpm_stream s,
                          qpm_run_handle *out);

/* A run whose fitness is the multi-wavelength objective o (fitness = -h;
 * cfg->fit_kernel is ignored, the DE shape is still tuned with cfg->tune).
 * o and its designs must outlive the run. Controls FIXED and DECAY (the
 * adaptive rule's thresholds are stated for |d_eff|^2: QPM_EINVAL);
 * qpm_run_polish is QPM_ENOTSUP on such a run. */
qpm_status qpm_run_create_objective(qpm_objective o, const qpm_run_config *cfg, qpm_stream s,
                                    qpm_run_handle *out);

/* Advance a run by `generations` (asynchronous on the run's stream; the
 * total may not exceed cfg->generations). */
qpm_status qpm_run_advance(qpm_run_handle r, int64_t generations);

/*
 * Copy the current state: x (device, np x ldx floats, may be NULL),
 * fitness (device, np floats or doubles per cfg->prec, may be NULL),
 * leaders (host int32[3], may be NULL: the leaders chosen in the last
 * completed generation, or at initialisation), *generation (host, may be
 * NULL). Synchronous.
 */
qpm_status qpm_run_read(qpm_run_handle r, float *x, int64_t ldx, void *fitness, int32_t *leaders,
                        int64_t *generation);

/* Best individual of the current population: best_x (device, D floats, may
 * be NULL), best_bits (device, W words, may be NULL), stats (host, may be
 * NULL). Synchronous. */
qpm_status qpm_run_best(qpm_run_handle r, float *best_x, uint32_t *best_bits, qpm_run_stats *stats);

/* F_g and a_g (host outputs, either may be NULL) of generation g, for
 * 0 <= g <= the generations completed (g < G): the values that generation
 * uses or used. Under QPM_CONTROL_ADAPTIVE, F_g exists once the population
 * entering g is known, so g past the completed count is QPM_EINVAL, as is
 * g >= G. Synchronous. */
qpm_status qpm_run_params(qpm_run_handle r, int64_t g, float *F, float *a);

/*
 * qpm_run_load -- replace the current population with caller genes x
 * (device, np x ldx floats, ldx >= D), then evaluate it and pick the
 * leaders again (a warm start from chosen designs, e.g. periodic poling).
 * The generation count is unchanged. Asynchronous on the run's stream.
 */
qpm_status qpm_run_load(qpm_run_handle r, const float *x, int64_t ldx);

/* Steps of one generation, in launch order (timing slots): the DE trials,
 * their evaluation, its finish (segment combine + selection + leaders),
 * the grey-wolf candidates, their evaluation, its finish (combine +
 * selection + next generation's DE draws + generation advance). */
enum {
    QPM_K_DE = 0,
    QPM_K_FIT_DE = 1,
    QPM_K_FINISH_DE = 2,
    QPM_K_GWO = 3,
    QPM_K_FIT_GWO = 4,
    QPM_K_FINISH_GWO = 5,
    QPM_K_COUNT = 6
};

/*
 * qpm_run_set_timing -- with enable != 0, qpm_run_advance launches each
 * generation kernel by kernel (no graph) on the run's stream with a HIP
 * event after every step, synchronises at the end of the call and adds the
 * measured durations to per-step totals; enable == 0 returns to the normal
 * mode. qpm_run_timing copies the totals (ms, host double[QPM_K_COUNT]) and
 * the number of timed generations, and with reset != 0 clears them.
 */
qpm_status qpm_run_set_timing(qpm_run_handle r, int32_t enable);
qpm_status qpm_run_timing(qpm_run_handle r, double *ms, int64_t *generations, int32_t reset);

/*
 * qpm_run_polish -- gradient polish of the three current leaders through the
 * relaxation (not in the paper): theta = the leader's genes, `steps` steps of
 * theta += eta g / max|g| with g = df/dtheta of qpm_relax_backward, then the
 * +-1 projection y = clamp(theta, -1, 1) (same signs) is scored by the exact
 * +-1 fitness and replaces the leader only if it is strictly better.
 * *accepted (host, may be NULL) receives how many of the three were
 * replaced. Synchronous; not captured in the generation graph.
 */
qpm_status qpm_run_polish(qpm_run_handle r, int32_t steps, float eta, int32_t *accepted);

/* Release a run (NULL accepted). */
qpm_status qpm_run_destroy(qpm_run_handle r);

/* qpm_run -- create, advance cfg->generations, report the best, destroy.
 * Synchronous. */
qpm_status qpm_run(qpm_design d, const qpm_run_config *cfg, float *best_x, uint32_t *best_bits,
                   qpm_run_stats *stats, qpm_stream s);

/*
 * Batches of independent designs (not in the paper, which optimises one
 * crystal per run): each step of a generation is one launch over all
 * instances. Instance b has N_b = offsets[b+1] - offsets[b] - 1 domains with
 * boundaries z[offsets[b] .. offsets[b+1]) (host, concatenated, offsets[0] =
 * 0) and mismatches dk1[b], dk2[b] (host). Its tables are those of
 * qpm_precompute_phases. Synchronises s. 1 <= n_inst <= 65535.
 */
qpm_status qpm_precompute_phases_batched(const double *z, const int64_t *offsets, int32_t n_inst,
                                         const double *dk1, const double *dk2, qpm_stream s,
                                         qpm_batch *out);
qpm_status qpm_batch_free(qpm_batch b);
/* n_inst, N_b (host int64[n_inst]) and C_b (host double[2 n_inst]); outputs
 * may be NULL. */
qpm_status qpm_batch_info(qpm_batch b, int32_t *n_inst, int64_t *n_domains, double *C);

/*
 * qpm_batch_eval_fitness -- f for np genomes of every instance. bits:
 * device, the population-major words of all instances stacked by instance
 * (sum_b W_b rows of ld words); fitness: device, n_inst x np floats / doubles
 * (instance-major). With waves_per_group = words_per_wave = 0 the
 * sign-pattern table kernel runs with its default shape; otherwise the
 * per-domain kernel with waves_per_group in {0 (default), 4, 8, 16} and
 * words_per_wave >= 0 (0 = default).
 */
qpm_status qpm_batch_eval_fitness(qpm_batch b, qpm_prec p, const uint32_t *bits, int64_t np,
                                  int64_t ld, void *fitness, int32_t waves_per_group,
                                  int32_t words_per_wave, qpm_stream s);

/*
 * qpm_batch_eval_fitness_table -- qpm_batch_eval_fitness with the table
 * kernel and an explicit shape: groups_per_workgroup in {1, 2, 4} groups of
 * 64 genomes x 4 waves, words_per_wave in [1, 5] (FP32) or [1, 2] (FP64).
 */
qpm_status qpm_batch_eval_fitness_table(qpm_batch b, qpm_prec p, const uint32_t *bits, int64_t np,
                                        int64_t ld, void *fitness, int32_t groups_per_workgroup,
                                        int32_t words_per_wave, qpm_stream s);

/*
 * qpm_batch_run_create -- one HWSDA run per instance, all advanced together
 * (every instance follows the single-design generation of qpm_run_create
 * with Philox instance number cfg->inst + b). 4 <= cfg->np <= 4096; the
 * fitness kernel is the batched sign-pattern table kernel of
 * qpm_batch_eval_fitness_table (cfg->fit_kernel is ignored). With tune != 0
 * its launch shape (genome groups per workgroup x words per wave) and the
 * DE shape are chosen by timing candidates on the initial population (kept
 * per problem size for the process, and appended to the file named by the
 * QPM_TUNE_CACHE environment variable if set).
 * Errors: QPM_EINVAL (NULL arguments, parameters out of range),
 * QPM_ERANGE (more than 65535 fitness segments or 1024-gene chunks over
 * the batch), QPM_ENOMEM, QPM_EHIP, QPM_ENOTSUP (not a gfx950 device).
 */
qpm_status qpm_batch_run_create(qpm_batch b, const qpm_run_config *cfg, int32_t tune, qpm_stream s,
                                qpm_batch_run_handle *out);
qpm_status qpm_batch_run_advance(qpm_batch_run_handle r, int64_t generations);
/* Launch shape of the batched DE step: individuals_per_wave in {1, 2, 4}
 * (gene chunks of 256 / individuals_per_wave) and passes in {1, 2, 4}
 * groups of individuals per workgroup; replaces the tuner's or default
 * choice (synchronises the run's stream and re-captures its graph). The
 * shape changes the speed only, never the trajectory. */
qpm_status qpm_batch_run_set_de_shape(qpm_batch_run_handle r, int32_t individuals_per_wave,
                                      int32_t passes);
qpm_status qpm_batch_run_set_timing(qpm_batch_run_handle r, int32_t enable);
qpm_status qpm_batch_run_timing(qpm_batch_run_handle r, double *ms, int64_t *generations,
                                int32_t reset);
/* State of instance inst: x (device np x ldx, ldx >= N_inst), fitness
 * (device np values), leaders (host int32[3]), fit_shape (host int32[2]:
 * waves per group, words per wave in use); any may be NULL. Synchronous. */
qpm_status qpm_batch_run_read(qpm_batch_run_handle r, int32_t inst, float *x, int64_t ldx,
                              void *fitness, int32_t *leaders, int32_t *fit_shape);
qpm_status qpm_batch_run_destroy(qpm_batch_run_handle r);

#ifdef __cplusplus
}
#endif

#endif /* QPM_H */
