// common.hpp -- shared host/device pieces of libqpm (HIP, gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdint>
#include <functional>
#include <string>

#include "qpm.h"

#define QPM_API extern "C" __attribute__((visibility("default")))

namespace qpm {

// ---------------------------------------------------------------- errors

void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

#define QPM_TRY_HIP(expr)                                                              \
    do {                                                                               \
        hipError_t qpm_e_ = (expr);                                                    \
        if (qpm_e_ != hipSuccess) {                                                    \
            ::qpm::set_error("%s failed: %s", #expr, hipGetErrorString(qpm_e_));     \
            return (qpm_e_ == hipErrorOutOfMemory) ? QPM_ENOMEM : QPM_EHIP;            \
        }                                                                              \
    } while (0)

#define QPM_REQUIRE(cond, code, ...)     \
    do {                                 \
        if (!(cond)) {                   \
            ::qpm::set_error(__VA_ARGS__); \
            return (code);               \
        }                                \
    } while (0)

// checks that the current device is gfx950
qpm_status check_device();

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
inline int64_t words_for(int64_t n) { return (n + 31) / 32; }

// ---------------------------------------------------------------- scratch

// Device scratch of an entry point (segment partials and the like) kept
// with a design or objective between calls instead of being allocated on
// every call. One buffer per stream, for up to kScratchSlots streams, found
// by the stream handle: work on one stream runs in order, so successive uses
// of a buffer never overlap, and the host lock is held from the lookup
// until the call's work has been enqueued, so threads sharing a stream do
// not interleave their launches. Calls under stream capture, or on more
// streams than there are slots, take their scratch from the stream-ordered
// allocator of their stream instead.
constexpr int kScratchSlots = 4;
struct ScratchCache;
ScratchCache *scratch_cache_create();
// synchronises the device (when a buffer exists), then frees the buffers
void scratch_cache_destroy(ScratchCache *c);

class ScratchLease {
public:
    ScratchLease(ScratchCache *c, hipStream_t s) : c_(c), s_(s) {}
    ~ScratchLease() { (void)end(); }
    ScratchLease(const ScratchLease &) = delete;
    ScratchLease &operator=(const ScratchLease &) = delete;
    // *p: at least `bytes` of device memory for work enqueued on s until end()
    qpm_status begin(size_t bytes, void **p);
    // after the work that uses the memory has been enqueued on s
    qpm_status end();

private:
    ScratchCache *c_;
    hipStream_t s_;
    void *owned_ = nullptr;
    bool locked_ = false;
};

// ---------------------------------------------------------------- design

struct Design {
    int64_t n = 0;       // domains
    int64_t words = 0;   // W = ceil(n / 32)
    double dk1 = 0, dk2 = 0;
    double C[2] = {0, 0};
    double4 *ph64 = nullptr;  // [32 W] {a.re, a.im, b.re, b.im}, zero padded
    float4 *ph32 = nullptr;   // [32 W] the same rounded to float
    double2 *c64 = nullptr;   // [n] diagonal terms c_n
    double *Cdev = nullptr;   // [2] C on the device
    double2 *tab64 = nullptr; // [8 W][A, B, Q][16 sign patterns] per 4-domain block
    int2 *tabq = nullptr;     // the same for the FP32 kernels: A and B as fixed-point
                              // integers at the word's scale, Q as float bits (word_tab_q)
    double *wsc = nullptr;    // [W] the word scales 2^-e_w of tabq (word_scales)
    int device = 0;
    double z0 = 0, zN = 0;    // first and last boundary
    uint64_t zhash = 0;       // FNV-1a of the boundary bytes (designs sharing z)
    ScratchCache *scratch = nullptr;  // per-call scratch of the entry points on this design
};

// Word scales of the fixed-point tables: for word w, sc[w] = 2^-e with e
// the largest integer such that M 2^e <= 2^31 - 64, M the sum of the word's
// domain widths (every |A| and |B| of a stretch of the word is at most the
// stretch's width sum, so the integer sums of a word stay below 2^31), with
// e at most 60. Host arrays: z[0..n], sc[ceil(n / 32)].
void word_scales(const double *z, int64_t n, double *sc);
// sign-pattern tables of the 8 W blocks of 4 domains (from ph64): tab64 in
// FP64, tabq in the fixed-point form at the scales wsc
qpm_status launch_pattern_tables(const double4 *ph64, int64_t words, const double *wsc, double2 *tab64, int2 *tabq,
                                 hipStream_t s);

// per-domain tables of one design into caller buffers (npad = 32 W
// entries of ph64 / ph32, n of c64) and C = sum c_n into Cdev[2]
qpm_status launch_phases(const double *zdev, int64_t n, double dk1, double dk2, double4 *ph64, float4 *ph32,
                         double2 *c64, double *Cdev, hipStream_t s);

// ---------------------------------------------------------------- fitness

struct FitPlan {
    int kind = QPM_FIT_SEGMENTED;  // qpm_fit_kernel (never AUTO here)
    int waves = 16;                // waves per workgroup (segmented) or genome groups (table)
    int wpw = 2;                   // bit words per wave
    int gy = 1;                    // workgroup segments along the domain axis
};

FitPlan plan_fitness(const Design &d, qpm_prec p, int64_t np, int kernel);
size_t fitness_workspace_bytes(const FitPlan &plan, int64_t ld);
qpm_status launch_fitness(const Design &d, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                          void *fitness, const FitPlan &plan, double *workspace, hipStream_t s);
// the segment triples only (6 x max(gy, 1) x ld doubles), for the fused
// finish step of a run
size_t fitness_partials_bytes(const FitPlan &plan, int64_t ld);
// advance (optional): the run's generation counter, incremented once by the
// kernel (which does not read it)
qpm_status launch_fitness_partials(const Design &d, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                   const FitPlan &plan, double *part, hipStream_t s, uint32_t *advance = nullptr);
// Finish one evaluation of a run: combine the triples of genome i into f,
// select (f > f_cur[i] replaces, leaders in skip3 excluded), then in a
// one-workgroup kernel: top3_out <- leaders (when non-null); with
// draws_next the DE draws of generation gen + 1 are written and gen is
// advanced.
// fbits (optional): packed copy of flags, 2 ceil(np / 64) words; cand:
// scratch of finish_cand_bytes(np) for the leader candidates (needed with
// top3_out)
// Selection outputs of a run without stored trials (all optional, together):
// the accepted slots appended to acc_list at *acc_cnt, and the packed flags
// from before the selection in fbits_prev.
struct AcceptOut {
    int32_t *list = nullptr;
    uint32_t *cnt = nullptr;
    uint32_t *fbits_prev = nullptr;
};
// How a finish step ends (defaults: as described at launch_finish):
// gen_advanced: the counter was already advanced by the evaluation kernel,
// so the next draws are for gen[0] itself and no tail advances it;
// defer_leaders: the candidates are left in `cand` for launch_materialize
// to merge into top3_out (no tail kernel); replace_all: every genome
// outside skip3 takes its new value (no greedy selection).
struct FinishMode {
    bool gen_advanced = false;
    bool defer_leaders = false;
    bool replace_all = false;
};
qpm_status launch_finish(const double *part, int gy, int64_t ld, int64_t np, const double *C, void *f_cur,
                         bool f64, uint32_t *flags, uint32_t *fbits, const int32_t *skip3, int32_t *top3_out,
                         void *cand, int4 *draws_next, uint32_t *gen, int64_t D, uint64_t seed, uint32_t inst,
                         hipStream_t s, AcceptOut acc = AcceptOut{}, FinishMode mode = FinishMode{});
inline size_t finish_cand_bytes(int64_t np)
{
    return static_cast<size_t>((np + 63) / 64) * 3 * (sizeof(double) + sizeof(int32_t));
}
// Adaptive F of the generation in the device counter g = gen[0] (nothing
// when g >= G): F_tab[g] from the statistics of f (np floats or doubles)
// and the decay law F_base[g]
qpm_status launch_adapt_F(const void *f, bool f64, int64_t np, const uint32_t *gen, int64_t G, const double *F_base,
                          float *F_tab, hipStream_t s);

// ---------------------------------------------------------------- multi-wavelength objective

constexpr int kMaxObjectiveDesigns = 8;

// per-design table pointers and C, passed by value to the kernels
struct ObjTabs {
    const int2 *tq[kMaxObjectiveDesigns];
    const double *wsc[kMaxObjectiveDesigns];
    const double2 *t64[kMaxObjectiveDesigns];
    double C[kMaxObjectiveDesigns][2];
};

// K designs on one set of boundaries; G_k = |A_k| / L (SHG) or
// |S_k| / L^2 (THG), fitness = -(sum |G0 - G_k| + beta (max G - min G))
struct Objective {
    const Design *d[kMaxObjectiveDesigns] = {};
    int K = 0;
    int kind = QPM_OBJ_SHG;
    double G0 = 1.0, beta = 0.0;
    double scale = 1.0;  // 1 / L or 1 / L^2
    int64_t n = 0, words = 0;
    ObjTabs tabs{};
    ScratchCache *scratch = nullptr;  // per-call scratch of the evaluation entry points
};

struct ObjPlan {
    int wpw = 1;  // bit words per segment wave (4 segment waves per workgroup)
    int gy = 1;   // workgroup segments along the domain axis
};

ObjPlan plan_objective(const Objective &o, qpm_prec p, int64_t np);
ObjPlan plan_objective_shape(const Objective &o, int wpw);
// segment partials of every design: K x gy x (6 or 2) x ld doubles
size_t objective_partials_bytes(const Objective &o, const ObjPlan &pl, int64_t ld);
qpm_status launch_objective_partials(const Objective &o, qpm_prec p, const uint32_t *bits, int64_t np, int64_t ld,
                                     const ObjPlan &pl, double *part, hipStream_t s, uint32_t *advance = nullptr);
// fitness (np floats or doubles) and optionally G ([K][ldG] doubles)
qpm_status launch_objective_values(const Objective &o, const ObjPlan &pl, const double *part, int64_t ld, int64_t np,
                                   void *fitness, bool f64, double *G, int64_t ldG, hipStream_t s);
// the run's finish step on the objective (as launch_finish)
qpm_status launch_objective_finish(const Objective &o, const ObjPlan &pl, const double *part, int64_t ld, int64_t np,
                                   void *f_cur, bool f64, uint32_t *flags, uint32_t *fbits, const int32_t *skip3,
                                   int32_t *top3_out, void *cand, int4 *draws_next, uint32_t *gen, int64_t D,
                                   uint64_t seed, uint32_t inst, hipStream_t s, AcceptOut acc = AcceptOut{},
                                   FinishMode mode = FinishMode{});

// ---------------------------------------------------------------- evolution kernels

// Rows of the current population live in one of two buffers; flags[i]
// (nullable = all 0) selects buf1 for row i. Trials / candidates of row i
// are written to the other buffer (out1 when flags is null).
struct PopView {
    const float *x0;
    const float *x1;
    const uint32_t *flags;
    float *out0;  // target of row i when flags[i] == 1
    float *out1;  // target of row i when flags[i] == 0 (or flags null)
    int64_t np, D, ldx;
};

qpm_status launch_init(int64_t np, int64_t D, int64_t ldx, uint64_t seed, uint32_t inst, float *x,
                       uint32_t *bits, int64_t ld, hipStream_t s);
// draws: device scratch of np int4 (donors r1, r2, r3 and jrand)
// Crossover threshold on a raw Philox word w: (w >> 8) 2^-24 <= CR holds
// exactly when (w >> 8) <= T = floor(CR 2^24) (CR 2^24 is exact), that is
// when w <= 256 T + 255.
inline uint32_t cr_threshold(float CR)
{
    const float t = std::floor(CR * 16777216.0f);
    if (t >= 16777215.0f) return 0xFFFFFFFFu;
    return static_cast<uint32_t>(t) * 256u + 255u;
}

// ipw: individuals per wave of the DE kernel (1, 2 or 4; 0 = chosen from np);
// passes: groups of individuals per workgroup (1, 2 or 4); fbits: optional
// packed copy of pv.flags (bit i % 32 of word i / 32)
qpm_status launch_de(const PopView &pv, float F, float CR, uint64_t seed, const uint32_t *gen_dev,
                     uint32_t gen, uint32_t inst, uint32_t *bits, int64_t ld, int4 *draws, bool compute_draws,
                     hipStream_t s, int ipw = 0, int passes = 1, const uint32_t *fbits = nullptr,
                     const float *F_tab = nullptr, bool store_genes = true, uint32_t *reset_cnt = nullptr);
// store_genes = false: the DE kernel writes the trials' bits only (and
// zeroes reset_cnt); launch_materialize then writes the genes of the
// accepted trials listed by the finish step (list, *cnt), reading the
// population before the selection through its packed flags fb_old
// (with top3_out: its first workgroup also merges the finish step's leader
// candidates, cand from a finish with defer_leaders, of ngroups groups)
qpm_status launch_materialize(const PopView &pv, const int4 *draws, const uint32_t *fb_old, float F,
                              const float *F_tab, float CR, uint64_t seed, const uint32_t *gen, uint32_t inst,
                              const int32_t *list, const uint32_t *cnt, hipStream_t s, const void *cand = nullptr,
                              int64_t ngroups = 0, bool f64 = false, int32_t *top3_out = nullptr);
// segmented plan with an explicit shape
FitPlan plan_fitness_shape(const Design &d, int waves, int wpw);
// table plan: gw genome groups of 64 per workgroup, wpw words per wave
// (1 <= wpw <= table_max_wpw: 4 wpw words of tables fit in 64 KB of LDS)
FitPlan plan_fitness_table(const Design &d, qpm_prec p, int gw, int wpw);
__host__ __device__ constexpr int table_max_wpw(bool f32) { return f32 ? 5 : 2; }
// LDS of one table-kernel workgroup (tables, reused for the combine)
size_t table_lds_bytes(int64_t W, bool f32, int gw, int wpw);
// DE draws of generation *gen_dev for every individual
qpm_status launch_draws(int64_t np, int64_t D, uint64_t seed, const uint32_t *gen_dev, uint32_t inst, int4 *draws,
                        hipStream_t s);
// leaders: device int32[3], or nullptr and the three by value in lead_c
qpm_status launch_gwo(const PopView &pv, const int32_t *leaders, const float *a_tab, float a,
                      uint64_t seed, const uint32_t *gen_dev, uint32_t gen, uint32_t inst,
                      int variant, uint32_t *bits, int64_t ld, hipStream_t s, int4 lead_c = int4{});
// the improved discrete four-leader step (leaders: 4 slots, the first three
// kept, on the device or by value in lead_c; par_tab[g] or
// par = {t, 1 - 2 eps, eps, lambda})
qpm_status launch_dgwo(const PopView &pv, const int32_t *leaders, const float4 *par_tab, float4 par,
                       uint64_t seed, const uint32_t *gen_dev, uint32_t gen, uint32_t inst, uint32_t *bits,
                       int64_t ld, hipStream_t s, int4 lead_c = int4{});
// leaders[3] = the best of f other than leaders[0..2]
qpm_status launch_fourth(const void *f, int64_t np, bool f64, int32_t *leaders, hipStream_t s);
// the three best of f[0..np) (f descending, slot ascending) into out3;
// T = float or double by `f64`
qpm_status launch_top3(const void *f, int64_t np, bool f64, int32_t *out3, hipStream_t s);
// rows of the current population (through flags) -> dense out[np][ldo]
qpm_status launch_gather(const PopView &pv, const int32_t *rows, int64_t nrows, float *out, int64_t ldo,
                         hipStream_t s);
// sign bits of every row of a dense population x[np][ldx] -> W x ld words
qpm_status launch_pack_pop(const float *x, int64_t np, int64_t D, int64_t ldx, uint32_t *bits, int64_t ld,
                           hipStream_t s);
// sign bits of one gene row (D genes) -> W words
qpm_status launch_pack_row(const float *x, int64_t D, uint32_t *bits, hipStream_t s);

// ---------------------------------------------------------------- fused generations

// Whole generations of a small population in one workgroup (fused.hip):
// both gene buffers, the fitness, bits, draws and (when they fit) the FP64
// tables in LDS. FP64 fitness, gwo_variant 0 or 1, any qpm_algo; F_g and a_g
// from the run's tables.
constexpr size_t kFusedMaxLds = 160 * 1024;
struct FusedRun {
    float *x0;
    const float *x1;
    uint32_t *flags, *fbits;
    void *f_cur;  // double, or float when f32
    int f32;
    int32_t *leaders;
    uint32_t *gen;
    const float *a_tab, *F_tab;
    const double2 *tab64;
    const double *C;
    int64_t np, D, ldx;
    float CR;
    uint64_t seed;
    uint32_t inst;
    int variant, algo;
};
// the population fits the kernel's LDS (np <= 64)
bool fused_eligible(int64_t np, int64_t D);
// gens generations from the run state (rows through flags, f, the counter);
// writes back every row to x0 with its flag cleared, f, the leaders of the
// last generation and the advanced counter
qpm_status launch_fused_generations(const FusedRun &fr, int gens, hipStream_t s);

// ---------------------------------------------------------------- polish

qpm_status launch_polish_step(float *theta, const float *grad, int64_t rows, int64_t n, int64_t ld, float eta,
                              hipStream_t s);
qpm_status launch_polish_project(const float *theta, float *y, int64_t rows, int64_t n, int64_t ld, hipStream_t s);
qpm_status launch_polish_accept(const float *y, int64_t n, int64_t ldy, const void *fcand, bool f64, const int32_t *L,
                                const PopView &pv, void *f_cur, uint32_t *accepted, hipStream_t s);

// ---------------------------------------------------------------- tuner cache

std::string tune_key(const char *kind, int64_t a, int64_t b, int prec, int64_t c);
// a cached shape, when present and accepted by `valid` (when given)
bool tune_lookup(const std::string &key, int *v0, int *v1,
                 const std::function<bool(int, int)> &valid = std::function<bool(int, int)>());
void tune_store(const std::string &key, int v0, int v1);

}  // namespace qpm

// The opaque handle types of the ABI are the library's structures.
struct qpm_design_s : public qpm::Design {};
struct qpm_objective_s : public qpm::Objective {};
