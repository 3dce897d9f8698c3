// run.hip -- the HWSDA loop on the device (paper Sec. 3.2, steps 1-7).
//
// State: genes in two buffers with a per-individual flag naming the buffer
// that holds the current row (selection flips a flag instead of copying a
// row); fitness of the current rows; one bit buffer reused for the DE
// trials and the GWO candidates; the leaders; a device generation counter
// and tables of a_g and F_g (the adaptive control writes F_g on the device
// once the population entering generation g is known). One generation is a fixed sequence of launches that
// reads g from the counter, so it is captured once into a HIP graph and
// replayed G times with no host work or synchronisation in between.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "common.hpp"

namespace qpm {

}  // namespace qpm

using namespace qpm;

struct qpm_run_s {
    const Design *d = nullptr;
    const Objective *obj = nullptr;  // multi-wavelength objective instead of |d_eff|^2
    ObjPlan oplan;
    qpm_run_config cfg{};
    hipStream_t st = nullptr;
    int64_t D = 0, ldx = 0, ld = 0, W = 0;
    float *buf[2] = {nullptr, nullptr};
    uint32_t *flags = nullptr;
    uint32_t *fbits = nullptr;  // flags packed one bit per individual (2 ceil(np / 64) words)
    void *cand = nullptr;       // leader candidates of the finish step (finish_cand_bytes)
    void *f_cur = nullptr;
    void *f_new = nullptr;
    uint32_t *tbits = nullptr;
    int32_t *leaders = nullptr;
    int32_t *best = nullptr;
    uint32_t *gen = nullptr;
    float *a_tab = nullptr;
    float *F_tab = nullptr;     // F_g per generation
    float4 *dg_tab = nullptr;   // discrete four-leader step: {t, 1 - 2 eps, eps, lambda} per generation
    double *F_base = nullptr;   // decay law of the adaptive control
    int4 *draws = nullptr;
    double *fws = nullptr;
    // trials not stored by the DE step: the accepted ones are listed by the
    // finish step and materialised afterwards (the DE step then writes bits
    // only, and the rejected majority costs no gene writes)
    bool lazy = false;
    int32_t *acc_list = nullptr;   // np slots
    uint32_t *acc_cnt = nullptr;
    uint32_t *fbits_prev = nullptr;  // packed flags before the selection
    FitPlan plan;
    int de_ipw = 0;     // 0 = chosen from np
    int de_passes = 1;  // groups of individuals per DE workgroup
    bool fused = false; // whole generations in one workgroup (fused.hip)
    hipGraph_t graph = nullptr;  // one generation
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph_k = nullptr;  // kGraphGens generations back to back
    hipGraphExec_t exec_k = nullptr;
    int64_t done = 0;
    // per-step timing (qpm_run_set_timing)
    bool timing = false;
    hipEvent_t ev[QPM_K_COUNT + 1] = {};
    double ms[QPM_K_COUNT] = {};
    int64_t timed = 0;
    // gradient polish of the leaders (qpm_run_polish), allocated on first use
    float *pol = nullptr;       // theta, grad, y: 3 rows of ldx each
    double *pol_S = nullptr;   // 3 x 2
    float *pol_f = nullptr;    // 3 relaxed values, then 3 ones (grad_f)
    void *pol_fc = nullptr;    // 3 exact fitness values
    uint32_t *pol_bits = nullptr;  // W x 64
    uint32_t *pol_acc = nullptr;
    double *pol_ws = nullptr;
    double *pol_edges = nullptr;  // relaxation edges of the 3 rows (both precisions' sizes)

    bool f64() const { return cfg.prec == QPM_PREC_F64; }
    bool adaptive() const { return cfg.control == QPM_CONTROL_ADAPTIVE; }
    PopView view() const { return PopView{buf[0], buf[1], flags, buf[0], buf[1], cfg.np, D, ldx}; }
};

static void release(qpm_run_s *r)
{
    if (!r) return;
    if (r->st) (void)hipStreamSynchronize(r->st);
    if (r->exec) (void)hipGraphExecDestroy(r->exec);
    if (r->graph) (void)hipGraphDestroy(r->graph);
    if (r->exec_k) (void)hipGraphExecDestroy(r->exec_k);
    if (r->graph_k) (void)hipGraphDestroy(r->graph_k);
    (void)hipFree(r->buf[0]);  // buf[1] lives in the same allocation
    (void)hipFree(r->flags);
    (void)hipFree(r->fbits);
    (void)hipFree(r->cand);
    (void)hipFree(r->f_cur);
    (void)hipFree(r->f_new);
    (void)hipFree(r->tbits);
    (void)hipFree(r->leaders);
    (void)hipFree(r->best);
    (void)hipFree(r->gen);
    (void)hipFree(r->a_tab);
    (void)hipFree(r->F_tab);
    (void)hipFree(r->dg_tab);
    (void)hipFree(r->F_base);
    (void)hipFree(r->fws);
    (void)hipFree(r->draws);
    (void)hipFree(r->acc_list);
    (void)hipFree(r->acc_cnt);
    (void)hipFree(r->fbits_prev);
    (void)hipFree(r->pol);
    (void)hipFree(r->pol_S);
    (void)hipFree(r->pol_f);
    (void)hipFree(r->pol_fc);
    (void)hipFree(r->pol_bits);
    (void)hipFree(r->pol_acc);
    (void)hipFree(r->pol_ws);
    (void)hipFree(r->pol_edges);
    for (auto &e : r->ev)
        if (e) (void)hipEventDestroy(e);
    if (r->st) (void)hipStreamDestroy(r->st);
    delete r;
}

// segment partials of the run's fitness for the genomes in tbits; with
// `advance` the kernel also advances the generation counter
static qpm_status eval_partials(qpm_run_s *r, uint32_t *advance = nullptr)
{
    const qpm_run_config &c = r->cfg;
    const qpm_prec p = static_cast<qpm_prec>(c.prec);
    if (r->obj)
        return launch_objective_partials(*r->obj, p, r->tbits, c.np, r->ld, r->oplan, r->fws, r->st, advance);
    return launch_fitness_partials(*r->d, p, r->tbits, c.np, r->ld, r->plan, r->fws, r->st, advance);
}

// combine + selection (+ leaders or the next generation's draws and advance)
static qpm_status eval_finish(qpm_run_s *r, const int32_t *skip3, int32_t *top3_out, void *cand, int4 *draws_next,
                              AcceptOut acc = AcceptOut{}, FinishMode mode = FinishMode{})
{
    const qpm_run_config &c = r->cfg;
    if (r->obj)
        return launch_objective_finish(*r->obj, r->oplan, r->fws, r->ld, c.np, r->f_cur, r->f64(), r->flags,
                                       r->fbits, skip3, top3_out, cand, draws_next, r->gen, r->D, c.seed, c.inst,
                                       r->st, acc, mode);
    const int gy = r->plan.kind == QPM_FIT_PER_GENOME ? 1 : r->plan.gy;
    return launch_finish(r->fws, gy, r->ld, c.np, r->d->Cdev, r->f_cur, r->f64(), r->flags, r->fbits, skip3,
                         top3_out, cand, draws_next, r->gen, r->D, c.seed, c.inst, r->st, acc, mode);
}

// the fitness of the genomes in tbits into f_cur (no selection)
static qpm_status eval_values(qpm_run_s *r)
{
    const qpm_run_config &c = r->cfg;
    const qpm_prec p = static_cast<qpm_prec>(c.prec);
    if (r->obj) {
        qpm_status st = launch_objective_partials(*r->obj, p, r->tbits, c.np, r->ld, r->oplan, r->fws, r->st);
        if (st != QPM_OK) return st;
        return launch_objective_values(*r->obj, r->oplan, r->fws, r->ld, c.np, r->f_cur, r->f64(), nullptr, 0, r->st);
    }
    return launch_fitness(*r->d, p, r->tbits, c.np, r->ld, r->f_cur, r->plan, r->fws, r->st);
}

// steps 2-6 for the generation held in the device counter; with `ev`, an
// event is recorded before each step and after the last
static qpm_status enqueue_generation(qpm_run_s *r, hipEvent_t *ev = nullptr)
{
    const qpm_run_config &c = r->cfg;
    const PopView pv = r->view();
    auto mark = [&](int k) -> qpm_status {
        if (ev) QPM_TRY_HIP(hipEventRecord(ev[k], r->st));
        return QPM_OK;
    };
    qpm_status st;
#define QPM_STEP(k, call)                         \
    if ((st = mark(k)) != QPM_OK) return st;      \
    if ((st = (call)) != QPM_OK) return st;
    if (c.algo == QPM_ALGO_DE) {
        // DE alone: trials, evaluation (which advances the counter), greedy
        // selection with the next generation's draws, and the three best
        // after it as the reported leaders
        QPM_STEP(QPM_K_DE, launch_de(pv, c.F, c.CR, c.seed, r->gen, 0u, c.inst, r->tbits, r->ld, r->draws, false,
                                     r->st, r->de_ipw, r->de_passes, r->fbits, r->F_tab, true, nullptr))
        QPM_STEP(QPM_K_FIT_DE, eval_partials(r, r->gen))
        QPM_STEP(QPM_K_FINISH_DE, eval_finish(r, nullptr, r->leaders, r->cand, r->draws, AcceptOut{},
                                              FinishMode{true, false, false}))
        if (r->adaptive()) {
            st = launch_adapt_F(r->f_cur, r->f64(), c.np, r->gen, c.generations, r->F_base, r->F_tab, r->st);
            if (st != QPM_OK) return st;
        }
        for (int k = QPM_K_GWO; k <= QPM_K_FINISH_GWO; ++k)
            if ((st = mark(k)) != QPM_OK) return st;
        return mark(QPM_K_COUNT);
    }
    if (c.algo == QPM_ALGO_GWO) {
        // GWO alone: the leaders are the three best of the population
        // entering the generation (from initialisation, or from the previous
        // generation's finish); every other wolf moves to its candidate
        for (int k = QPM_K_DE; k <= QPM_K_FINISH_DE; ++k)
            if ((st = mark(k)) != QPM_OK) return st;
        if (c.gwo_variant == 2) {
            QPM_STEP(QPM_K_GWO, launch_fourth(r->f_cur, c.np, r->f64(), r->leaders, r->st))
            st = launch_dgwo(pv, r->leaders, r->dg_tab, float4{}, c.seed, r->gen, 0u, c.inst, r->tbits, r->ld,
                             r->st);
            if (st != QPM_OK) return st;
        } else {
            QPM_STEP(QPM_K_GWO, launch_gwo(pv, r->leaders, r->a_tab, 0.0f, c.seed, r->gen, 0u, c.inst,
                                           c.gwo_variant, r->tbits, r->ld, r->st))
        }
        QPM_STEP(QPM_K_FIT_GWO, eval_partials(r, r->gen))
        // leaders kept; the next leaders from the moved population
        QPM_STEP(QPM_K_FINISH_GWO, eval_finish(r, r->leaders, r->leaders, r->cand, nullptr, AcceptOut{},
                                               FinishMode{true, false, true}))
        if (r->adaptive()) {
            st = launch_adapt_F(r->f_cur, r->f64(), c.np, r->gen, c.generations, r->F_base, r->F_tab, r->st);
            if (st != QPM_OK) return st;
        }
        return mark(QPM_K_COUNT);
    }
    QPM_STEP(QPM_K_DE, launch_de(pv, c.F, c.CR, c.seed, r->gen, 0u, c.inst, r->tbits, r->ld, r->draws, false, r->st,
                                 r->de_ipw, r->de_passes, r->fbits, r->F_tab, !r->lazy,
                                 r->lazy ? r->acc_cnt : nullptr))
    QPM_STEP(QPM_K_FIT_DE, eval_partials(r))
    // with accepted-only trials the materialise kernel also merges the
    // leader candidates (no separate one-workgroup kernel)
    QPM_STEP(QPM_K_FINISH_DE, eval_finish(r, nullptr, r->leaders, r->cand, nullptr,
                                          r->lazy ? AcceptOut{r->acc_list, r->acc_cnt, r->fbits_prev} : AcceptOut{},
                                          FinishMode{false, r->lazy}))
    if (r->lazy) {  // the accepted trials' genes (timed with the finish)
        st = launch_materialize(pv, r->draws, r->fbits_prev, c.F, r->F_tab, c.CR, c.seed, r->gen, c.inst,
                                r->acc_list, r->acc_cnt, r->st, r->cand, (c.np + 63) / 64, r->f64(), r->leaders);
        if (st != QPM_OK) return st;
    }
    if (c.gwo_variant == 2) {
        // the fourth leader (after DE selection), then the discrete step
        QPM_STEP(QPM_K_GWO, launch_fourth(r->f_cur, c.np, r->f64(), r->leaders, r->st))
        st = launch_dgwo(pv, r->leaders, r->dg_tab, float4{}, c.seed, r->gen, 0u, c.inst, r->tbits, r->ld, r->st);
        if (st != QPM_OK) return st;
    } else {
        QPM_STEP(QPM_K_GWO, launch_gwo(pv, r->leaders, r->a_tab, 0.0f, c.seed, r->gen, 0u, c.inst, c.gwo_variant,
                                       r->tbits, r->ld, r->st))
    }
    // the evaluation kernel advances the generation counter (it does not
    // read it), so the finish step needs no one-workgroup kernel after it
    QPM_STEP(QPM_K_FIT_GWO, eval_partials(r, r->gen))
    QPM_STEP(QPM_K_FINISH_GWO, eval_finish(r, r->leaders, nullptr, nullptr, r->draws, AcceptOut{},
                                           FinishMode{true, false}))
    if (r->adaptive()) {  // F of the next generation (timed with the finish)
        st = launch_adapt_F(r->f_cur, r->f64(), c.np, r->gen, c.generations, r->F_base, r->F_tab, r->st);
        if (st != QPM_OK) return st;
    }
#undef QPM_STEP
    return mark(QPM_K_COUNT);
}

// Capture `gens` generations (each reads g from the device counter) into
// one graph; advancing by whole multiples of kGraphGens replays the long
// graph, which saves the gaps between graph launches.
constexpr int64_t kGraphGens = 8;

static qpm_status capture_generations(qpm_run_s *r, int64_t gens, hipGraph_t *graph, hipGraphExec_t *exec)
{
    hipError_t e = hipStreamBeginCapture(r->st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        set_error("hipStreamBeginCapture failed: %s", hipGetErrorString(e));
        return QPM_EHIP;
    }
    qpm_status st = QPM_OK;
    for (int64_t g = 0; g < gens && st == QPM_OK; ++g) st = enqueue_generation(r);
    e = hipStreamEndCapture(r->st, graph);
    if (st == QPM_OK && e != hipSuccess) {
        set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
        st = QPM_EHIP;
    }
    if (st == QPM_OK) {
        e = hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            set_error("hipGraphInstantiate failed: %s", hipGetErrorString(e));
            st = QPM_EHIP;
        }
    }
    return st;
}

// Time candidate launch shapes on the initial population (bits in tbits,
// genes in buf[0]) and keep the fastest: the segmented fitness shape
// (waves per workgroup, words per wave) and the DE chunk width (individuals
// per wave). Every candidate computes the same values (the fitness up to the
// summation order). Leaves buf[1], tbits and draws overwritten.
static qpm_status tune_run(qpm_run_s *r)
{
    const qpm_run_config &c = r->cfg;
    const qpm_prec p = static_cast<qpm_prec>(c.prec);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    QPM_TRY_HIP(hipEventCreate(&e0));
    QPM_TRY_HIP(hipEventCreate(&e1));
    // the fastest of five single launches after a warm-up (the minimum is
    // the estimate least disturbed by other work on the device)
    auto time_min = [&](auto &&launch, float *ms) -> qpm_status {
        qpm_status st = launch();
        *ms = 1e30f;
        for (int rep = 0; rep < 5 && st == QPM_OK; ++rep) {
            QPM_TRY_HIP(hipEventRecord(e0, r->st));
            st = launch();
            QPM_TRY_HIP(hipEventRecord(e1, r->st));
            QPM_TRY_HIP(hipEventSynchronize(e1));
            float t = 0.0f;
            QPM_TRY_HIP(hipEventElapsedTime(&t, e0, e1));
            if (t < *ms) *ms = t;
        }
        return st;
    };
    qpm_status st = QPM_OK;
    if (r->obj) {
        // words per wave of the objective kernel (partials + values)
        const Objective &o = *r->obj;
        const std::string key = tune_key(o.kind == QPM_OBJ_THG ? "objthg" : "objshg", o.words * 16 + o.K, c.np,
                                         c.prec, 1);
        int wpw = 0, unused = 0;
        const int maxw = table_max_wpw(p == QPM_PREC_F32);
        if (!tune_lookup(key, &wpw, &unused,
                         [&](int w, int) { return w >= 1 && w <= maxw && plan_objective_shape(o, w).gy <= 65535; })) {
            std::vector<ObjPlan> cands;
            for (int w = 1; w <= table_max_wpw(p == QPM_PREC_F32); ++w) {
                const ObjPlan pl = plan_objective_shape(o, w);
                if (pl.gy <= 65535) cands.push_back(pl);
            }
            size_t maxb = 0;
            for (const auto &pl : cands) maxb = std::max(maxb, objective_partials_bytes(o, pl, r->ld));
            double *part = nullptr;
            QPM_TRY_HIP(hipMallocAsync(reinterpret_cast<void **>(&part), maxb, r->st));
            float best = 1e30f;
            for (const auto &pl : cands) {
                float ms = 0.0f;
                st = time_min(
                    [&]() {
                        qpm_status s2 = launch_objective_partials(o, p, r->tbits, c.np, r->ld, pl, part, r->st);
                        if (s2 != QPM_OK) return s2;
                        return launch_objective_values(o, pl, part, r->ld, c.np, r->f_new, r->f64(), nullptr, 0,
                                                       r->st);
                    },
                    &ms);
                if (st != QPM_OK) break;
                if (ms < best) {
                    best = ms;
                    wpw = pl.wpw;
                }
            }
            (void)hipFreeAsync(part, r->st);
            if (st != QPM_OK) return st;
            tune_store(key, wpw, 0);
        }
        r->oplan = plan_objective_shape(o, wpw);
    } else if (r->plan.kind == QPM_FIT_SEGMENTED) {
        const std::string key = tune_key("fit", r->d->words, c.np, c.prec, 1);
        int waves = 0, wpw = 0;
        const auto seg_ok = [&](int wv, int w) {
            return (wv == 1 || wv == 2 || wv == 4 || wv == 8 || wv == 16) && w >= 1 &&
                   plan_fitness_shape(*r->d, wv, w).gy <= 65535;
        };
        if (!tune_lookup(key, &waves, &wpw, seg_ok)) {
            const int w0 = r->plan.wpw;
            std::vector<FitPlan> cands;
            for (int wv : {4, 8, 16})
                for (int f : {1, 2, 4, 8}) {
                    FitPlan pl = plan_fitness_shape(*r->d, wv, std::max(1, w0 * f / 2));
                    if (pl.gy <= 65535) cands.push_back(pl);
                }
            size_t maxb = 0;
            for (const auto &pl : cands) maxb = std::max(maxb, fitness_partials_bytes(pl, r->ld));
            double *part = nullptr;
            QPM_TRY_HIP(hipMallocAsync(reinterpret_cast<void **>(&part), maxb, r->st));
            // a candidate is timed with its segment combine (the run's finish
            // step does the same combine), so more segments are not free
            float best = 1e30f;
            for (const auto &pl : cands) {
                float ms = 0.0f;
                st = time_min(
                    [&]() { return launch_fitness(*r->d, p, r->tbits, c.np, r->ld, r->f_new, pl, part, r->st); },
                    &ms);
                if (st != QPM_OK) break;
                if (ms < best) {
                    best = ms;
                    waves = pl.waves;
                    wpw = pl.wpw;
                }
            }
            (void)hipFreeAsync(part, r->st);
            if (st != QPM_OK) return st;
            tune_store(key, waves, wpw);
        }
        r->plan = plan_fitness_shape(*r->d, waves, wpw);
    } else if (r->plan.kind == QPM_FIT_TABLE) {
        const std::string key = tune_key("tab", r->d->words, c.np, c.prec, 1);
        int gw = 0, wpw = 0;
        const auto tab_ok = [&](int g, int w) {
            return (g == 1 || g == 2 || g == 4) && w >= 1 && w <= table_max_wpw(p == QPM_PREC_F32) &&
                   plan_fitness_table(*r->d, p, g, w).gy <= 65535;
        };
        if (!tune_lookup(key, &gw, &wpw, tab_ok)) {
            std::vector<FitPlan> cands;
            for (int g : {1, 2, 4})
                for (int w = 1; w <= table_max_wpw(p == QPM_PREC_F32); ++w) {
                    FitPlan pl = plan_fitness_table(*r->d, p, g, w);
                    if (pl.gy <= 65535) cands.push_back(pl);
                }
            size_t maxb = 0;
            for (const auto &pl : cands) maxb = std::max(maxb, fitness_partials_bytes(pl, r->ld));
            double *part = nullptr;
            QPM_TRY_HIP(hipMallocAsync(reinterpret_cast<void **>(&part), maxb, r->st));
            float best = 1e30f;
            for (const auto &pl : cands) {
                float ms = 0.0f;
                st = time_min(
                    [&]() { return launch_fitness(*r->d, p, r->tbits, c.np, r->ld, r->f_new, pl, part, r->st); },
                    &ms);
                if (st != QPM_OK) break;
                if (ms < best) {
                    best = ms;
                    gw = pl.waves;
                    wpw = pl.wpw;
                }
            }
            (void)hipFreeAsync(part, r->st);
            if (st != QPM_OK) return st;
            tune_store(key, gw, wpw);
        }
        r->plan = plan_fitness_table(*r->d, p, gw, wpw);
    }
    {
        const std::string key = tune_key("de2", r->D, c.np, 0, 1);
        int ipw = 0, passes = 0;
        const auto de_ok = [](int w, int pc) { return (w == 1 || w == 2 || w == 4) && (pc == 1 || pc == 2 || pc == 4); };
        if (!tune_lookup(key, &ipw, &passes, de_ok)) {
            st = launch_draws(c.np, r->D, c.seed, r->gen, c.inst, r->draws, r->st);
            if (st != QPM_OK) return st;
            const PopView pv = r->view();
            float best = 1e30f;
            for (int cand : {1, 2, 4})
                for (int np_ : {1, 2, 4}) {
                    float ms = 0.0f;
                    st = time_min([&]() {
                        return launch_de(pv, c.F, c.CR, c.seed, r->gen, 0u, c.inst, r->tbits, r->ld, r->draws, false,
                                         r->st, cand, np_, r->fbits, nullptr, !r->lazy, nullptr);
                    },
                               &ms);
                    if (st != QPM_OK) return st;
                    if (ms < best) {
                        best = ms;
                        ipw = cand;
                        passes = np_;
                    }
                }
            tune_store(key, ipw, passes);
        }
        r->de_ipw = ipw;
        r->de_passes = passes >= 1 ? passes : 1;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return QPM_OK;
}

static qpm_status create_run(const Design *d, const Objective *obj, const qpm_run_config *cfg, qpm_stream sv,
                             qpm_run_handle *out)
{
    QPM_REQUIRE(d && cfg && out, QPM_EINVAL, "design, cfg and out must not be NULL");
    const qpm_run_config c = *cfg;
    QPM_REQUIRE(c.np >= 4 && c.np <= (int64_t(1) << 24), QPM_EINVAL, "np must be in [4, 2^24] (got %lld)",
                (long long)c.np);
    QPM_REQUIRE(c.generations >= 1 && c.generations <= (int64_t(1) << 31) - 2, QPM_EINVAL,
                "generations must be in [1, 2^31 - 2]");
    QPM_REQUIRE(c.F >= 0.0f && c.F <= 2.0f, QPM_EINVAL, "F must be in [0, 2] (got %g)", (double)c.F);
    QPM_REQUIRE(c.CR >= 0.0f && c.CR <= 1.0f, QPM_EINVAL, "CR must be in [0, 1] (got %g)", (double)c.CR);
    QPM_REQUIRE(c.prec == QPM_PREC_F32 || c.prec == QPM_PREC_F64, QPM_EINVAL, "unknown precision %d", c.prec);
    QPM_REQUIRE(c.gwo_variant >= 0 && c.gwo_variant <= 2, QPM_EINVAL, "gwo_variant must be 0, 1 or 2");
    QPM_REQUIRE(c.inst < (1u << 24), QPM_EINVAL, "inst must be < 2^24");
    QPM_REQUIRE(c.fit_kernel == QPM_FIT_AUTO || c.fit_kernel == QPM_FIT_SEGMENTED ||
                    c.fit_kernel == QPM_FIT_PER_GENOME || c.fit_kernel == QPM_FIT_TABLE,
                QPM_EINVAL, "unknown fitness kernel %d", c.fit_kernel);
    QPM_REQUIRE(!(c.fit_kernel == QPM_FIT_PER_GENOME && c.prec != QPM_PREC_F64), QPM_EINVAL,
                "the per-genome kernel computes in FP64 only");
    QPM_REQUIRE(c.control == QPM_CONTROL_FIXED || c.control == QPM_CONTROL_DECAY ||
                    c.control == QPM_CONTROL_ADAPTIVE,
                QPM_EINVAL, "unknown parameter control %d", c.control);
    QPM_REQUIRE(c.trials == QPM_TRIALS_AUTO || c.trials == QPM_TRIALS_STORE || c.trials == QPM_TRIALS_ACCEPTED,
                QPM_EINVAL, "unknown trial storage %d", c.trials);
    QPM_REQUIRE(c.algo == QPM_ALGO_HWSDA || c.algo == QPM_ALGO_DE || c.algo == QPM_ALGO_GWO, QPM_EINVAL,
                "unknown algorithm %d", c.algo);
    QPM_REQUIRE(c.algo == QPM_ALGO_HWSDA || c.trials != QPM_TRIALS_ACCEPTED, QPM_EINVAL,
                "accepted-only trials are a mode of the hybrid run; DE and GWO runs store every trial");
    QPM_REQUIRE(c.fused >= -1 && c.fused <= 1, QPM_EINVAL, "fused must be -1, 0 or 1 (got %d)", (int)c.fused);
    const bool fused_ok = obj == nullptr &&
                          (c.fit_kernel == QPM_FIT_AUTO || c.fit_kernel == QPM_FIT_TABLE) &&
                          c.control != QPM_CONTROL_ADAPTIVE && (c.gwo_variant == 0 || c.gwo_variant == 1) &&
                          fused_eligible(c.np, d->n);
    QPM_REQUIRE(c.fused != 1 || fused_ok, QPM_ENOTSUP,
                "fused generations need table fitness, a fixed or decaying control, gwo_variant 0 or 1, no "
                "objective and a population that fits in LDS (np <= 64)");
    qpm_status st = check_device();
    if (st != QPM_OK) return st;

    auto *r = new qpm_run_s();
    r->d = d;
    r->obj = obj;
    r->cfg = c;
    r->D = d->n;
    r->ldx = ((r->D + 63) / 64) * 64;
    r->ld = ((c.np + 63) / 64) * 64;
    r->W = d->words;
    // trials are materialised only for the accepted ones when the two gene
    // buffers are large: every stored trial costs write bandwidth (HBM once
    // the population spills the 256 MB last-level cache), while
    // recomputing an accepted one
    // reads four rows; below about 64 MB of population (both buffers) the
    // stored trials cost less (measured, whole runs: 82-329 MB populations
    // gain 4-6 % with accepted-only trials, 16-33 MB ones lose 2-6 %, 41 MB
    // is even)
    const bool lazy_ok = c.np <= 65536 && r->ldx < (int64_t(1) << 24);
    if (c.trials == QPM_TRIALS_ACCEPTED && !lazy_ok) {
        set_error("materialising accepted trials needs np <= 65536");
        release(r);
        return QPM_EINVAL;
    }
    r->fused = fused_ok && c.fused != -1;
    r->lazy = c.trials == QPM_TRIALS_ACCEPTED ||
              (c.trials == QPM_TRIALS_AUTO && c.algo == QPM_ALGO_HWSDA && lazy_ok &&
               2 * static_cast<int64_t>(sizeof(float)) * c.np * r->ldx > (int64_t(64) << 20));
    r->plan = plan_fitness(*d, static_cast<qpm_prec>(c.prec), c.np, c.fit_kernel);
    if (obj) r->oplan = plan_objective(*obj, static_cast<qpm_prec>(c.prec), c.np);
    const size_t es = r->f64() ? sizeof(double) : sizeof(float);
    const size_t gene_bytes = sizeof(float) * static_cast<size_t>(c.np) * static_cast<size_t>(r->ldx);
    hipError_t e = hipStreamCreateWithFlags(&r->st, hipStreamNonBlocking);
    // both gene buffers in one allocation (buf[1] = buf[0] + np ldx), so
    // the DE kernel can address row r of either buffer as one array
    if (e == hipSuccess) e = hipMalloc(&r->buf[0], 2 * gene_bytes);
    if (e == hipSuccess) r->buf[1] = r->buf[0] + c.np * r->ldx;
    if (e == hipSuccess) e = hipMalloc(&r->flags, sizeof(uint32_t) * c.np);
    if (e == hipSuccess) e = hipMalloc(&r->fbits, sizeof(uint32_t) * 2 * ((c.np + 63) / 64));
    if (e == hipSuccess) e = hipMalloc(&r->cand, finish_cand_bytes(c.np));
    if (e == hipSuccess) e = hipMalloc(&r->f_cur, es * c.np);
    if (e == hipSuccess) e = hipMalloc(&r->f_new, es * c.np);
    if (e == hipSuccess) e = hipMalloc(&r->tbits, sizeof(uint32_t) * r->W * r->ld);
    if (e == hipSuccess) e = hipMalloc(&r->leaders, sizeof(int32_t) * 4);  // the fourth for variant 2
    if (e == hipSuccess) e = hipMalloc(&r->best, sizeof(int32_t) * 3);
    if (e == hipSuccess) e = hipMalloc(&r->gen, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&r->a_tab, sizeof(float) * c.generations);
    if (e == hipSuccess) e = hipMalloc(&r->F_tab, sizeof(float) * c.generations);
    if (e == hipSuccess && r->adaptive()) e = hipMalloc(&r->F_base, sizeof(double) * c.generations);
    if (e == hipSuccess && c.gwo_variant == 2) e = hipMalloc(&r->dg_tab, sizeof(float4) * c.generations);
    if (e == hipSuccess) e = hipMalloc(&r->draws, sizeof(int4) * c.np);
    if (e == hipSuccess && r->lazy) e = hipMalloc(&r->acc_list, sizeof(int32_t) * c.np);
    if (e == hipSuccess && r->lazy) e = hipMalloc(&r->acc_cnt, sizeof(uint32_t));
    if (e == hipSuccess && r->lazy) e = hipMalloc(&r->fbits_prev, sizeof(uint32_t) * 2 * ((c.np + 63) / 64));
    if (e != hipSuccess) {
        set_error("run allocation failed: %s", hipGetErrorString(e));
        release(r);
        return e == hipErrorOutOfMemory ? QPM_ENOMEM : QPM_EHIP;
    }
    // a_g and F_g per control, evaluated in double with t = g / G:
    // fixed: a_g = 2 (1 - t) and F_g = F; decay: F_g = a_g = 0.1 (1 - t) +
    // 0.01 t; adaptive: a_g as in decay, F_g written on the device from the
    // decay law base(g) = 0.1 (cos(pi t / 2) + 1) / 2 (1 - 0.2 t^2)
    std::vector<float> a(c.generations), F(c.generations);
    std::vector<double> base(r->adaptive() ? c.generations : 0);
    // discrete four-leader step: t, 1 - 2 eps, eps = 0.1 (1 - t) + 0.01 t,
    // lambda = 0.2 (1 - t), each rounded to float once
    std::vector<float4> dg(c.gwo_variant == 2 ? c.generations : 0);
    for (int64_t g = 0; g < c.generations; ++g) {
        const double t = static_cast<double>(g) / static_cast<double>(c.generations);
        if (c.control == QPM_CONTROL_FIXED) {
            a[g] = static_cast<float>(2.0 * (1.0 - t));
            F[g] = c.F;
        } else {
            a[g] = static_cast<float>(0.1 * (1.0 - t) + 0.01 * t);
            F[g] = a[g];
        }
        if (r->adaptive()) base[g] = 0.1 * (0.5 * (std::cos(0.5 * M_PI * t) + 1.0)) * (1.0 - 0.2 * t * t);
        if (c.gwo_variant == 2) {
            const float eps = static_cast<float>(0.1 * (1.0 - t) + 0.01 * t);
            dg[g] = make_float4(static_cast<float>(t), static_cast<float>(1.0 - 2.0 * static_cast<double>(eps)), eps,
                                static_cast<float>(0.2 * (1.0 - t)));
        }
    }

    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, static_cast<hipStream_t>(sv));
    if (e == hipSuccess) e = hipStreamWaitEvent(r->st, ev, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(r->a_tab, a.data(), sizeof(float) * c.generations, hipMemcpyHostToDevice, r->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(r->F_tab, F.data(), sizeof(float) * c.generations, hipMemcpyHostToDevice, r->st);
    if (e == hipSuccess && r->adaptive())
        e = hipMemcpyAsync(r->F_base, base.data(), sizeof(double) * c.generations, hipMemcpyHostToDevice, r->st);
    if (e == hipSuccess && c.gwo_variant == 2)
        e = hipMemcpyAsync(r->dg_tab, dg.data(), sizeof(float4) * c.generations, hipMemcpyHostToDevice, r->st);
    if (e == hipSuccess) e = hipMemsetAsync(r->flags, 0, sizeof(uint32_t) * c.np, r->st);
    if (e == hipSuccess) e = hipMemsetAsync(r->fbits, 0, sizeof(uint32_t) * 2 * ((c.np + 63) / 64), r->st);
    if (e == hipSuccess) e = hipMemsetAsync(r->gen, 0, sizeof(uint32_t), r->st);
    if (e == hipSuccess && r->lazy) e = hipMemsetAsync(r->acc_cnt, 0, sizeof(uint32_t), r->st);
    if (e == hipSuccess) e = hipMemsetAsync(r->tbits, 0, sizeof(uint32_t) * r->W * r->ld, r->st);
    if (e == hipSuccess) e = hipMemsetAsync(r->buf[1], 0, gene_bytes, r->st);
    if (e == hipSuccess) e = hipStreamSynchronize(r->st);  // the host tables must outlive the copies
    if (ev) (void)hipEventDestroy(ev);
    if (e != hipSuccess) {
        set_error("run set-up failed: %s", hipGetErrorString(e));
        release(r);
        return QPM_EHIP;
    }
    // step 1: initialise, evaluate, leaders (after tuning on the initial
    // population, which the tuner's trial launches overwrite)
    st = launch_init(c.np, r->D, r->ldx, c.seed, c.inst, r->buf[0], r->tbits, r->ld, r->st);
    if (st == QPM_OK && c.tune) {
        st = tune_run(r);
        if (st == QPM_OK) st = launch_init(c.np, r->D, r->ldx, c.seed, c.inst, r->buf[0], r->tbits, r->ld, r->st);
    }
    if (st == QPM_OK) {
        e = hipMalloc(&r->fws, obj ? objective_partials_bytes(*obj, r->oplan, r->ld)
                                   : fitness_partials_bytes(r->plan, r->ld));
        if (e != hipSuccess) {
            set_error("run allocation failed: %s", hipGetErrorString(e));
            st = e == hipErrorOutOfMemory ? QPM_ENOMEM : QPM_EHIP;
        }
    }
    if (st == QPM_OK) st = eval_values(r);
    if (st == QPM_OK) st = launch_top3(r->f_cur, c.np, r->f64(), r->leaders, r->st);
    if (st == QPM_OK) st = launch_draws(c.np, r->D, c.seed, r->gen, c.inst, r->draws, r->st);
    if (st == QPM_OK && r->adaptive())
        st = launch_adapt_F(r->f_cur, r->f64(), c.np, r->gen, c.generations, r->F_base, r->F_tab, r->st);
    if (st == QPM_OK && c.use_graph && !r->fused) {
        st = capture_generations(r, 1, &r->graph, &r->exec);
        if (st == QPM_OK && c.generations >= 2 * kGraphGens)
            st = capture_generations(r, kGraphGens, &r->graph_k, &r->exec_k);
    }
    if (st != QPM_OK) {
        release(r);
        return st;
    }
    *out = r;
    return QPM_OK;
}

QPM_API qpm_status qpm_run_create(qpm_design d, const qpm_run_config *cfg, qpm_stream sv, qpm_run_handle *out)
{
    clear_error();
    return create_run(d, nullptr, cfg, sv, out);
}

QPM_API qpm_status qpm_run_create_objective(qpm_objective o, const qpm_run_config *cfg, qpm_stream sv,
                                            qpm_run_handle *out)
{
    clear_error();
    QPM_REQUIRE(o != nullptr && cfg != nullptr, QPM_EINVAL, "objective and cfg must not be NULL");
    QPM_REQUIRE(cfg->control != QPM_CONTROL_ADAPTIVE, QPM_EINVAL,
                "the adaptive control is defined for the |d_eff|^2 fitness, not for the objective");
    return create_run(o->d[0], o, cfg, sv, out);
}

QPM_API qpm_status qpm_run_advance(qpm_run_handle r, int64_t generations)
{
    clear_error();
    QPM_REQUIRE(r != nullptr, QPM_EINVAL, "run is NULL");
    QPM_REQUIRE(generations >= 0 && r->done + generations <= r->cfg.generations, QPM_EINVAL,
                "advancing %lld generations would pass the configured %lld (done %lld)", (long long)generations,
                (long long)r->cfg.generations, (long long)r->done);
    int64_t g = 0;
    if (!r->timing && r->fused && generations > 0) {
        // whole generations in one workgroup, in launches of at most 1000
        const qpm_run_config &c = r->cfg;
        FusedRun fr{r->buf[0], r->buf[1], r->flags, r->fbits, r->f_cur, c.prec == QPM_PREC_F32, r->leaders, r->gen,
                    r->a_tab, r->F_tab, r->d->tab64, r->d->Cdev, c.np, r->D, r->ldx, c.CR, c.seed, c.inst,
                    c.gwo_variant, c.algo};
        for (; g < generations;) {
            const int k = static_cast<int>(std::min<int64_t>(1000, generations - g));
            qpm_status st = launch_fused_generations(fr, k, r->st);
            if (st != QPM_OK) return st;
            g += k;
            r->done += k;
        }
        // the DE draws of the coming generation, for the multi-kernel path
        return launch_draws(c.np, r->D, c.seed, r->gen, c.inst, r->draws, r->st);
    }
    if (!r->timing && r->exec_k)
        for (; g + kGraphGens <= generations; g += kGraphGens) {
            QPM_TRY_HIP(hipGraphLaunch(r->exec_k, r->st));
            r->done += kGraphGens;
        }
    for (; g < generations; ++g) {
        if (r->timing) {
            qpm_status st = enqueue_generation(r, r->ev);
            if (st != QPM_OK) return st;
            QPM_TRY_HIP(hipEventSynchronize(r->ev[QPM_K_COUNT]));
            for (int k = 0; k < QPM_K_COUNT; ++k) {
                float t = 0.0f;
                QPM_TRY_HIP(hipEventElapsedTime(&t, r->ev[k], r->ev[k + 1]));
                r->ms[k] += t;
            }
            ++r->timed;
        } else if (r->exec) {
            QPM_TRY_HIP(hipGraphLaunch(r->exec, r->st));
        } else {
            qpm_status st = enqueue_generation(r);
            if (st != QPM_OK) return st;
        }
        ++r->done;
    }
    return QPM_OK;
}

QPM_API qpm_status qpm_run_set_timing(qpm_run_handle r, int32_t enable)
{
    clear_error();
    QPM_REQUIRE(r != nullptr, QPM_EINVAL, "run is NULL");
    if (enable && !r->ev[0])
        for (auto &e : r->ev) QPM_TRY_HIP(hipEventCreate(&e));
    r->timing = enable != 0;
    return QPM_OK;
}

QPM_API qpm_status qpm_run_timing(qpm_run_handle r, double *ms, int64_t *generations, int32_t reset)
{
    clear_error();
    QPM_REQUIRE(r != nullptr, QPM_EINVAL, "run is NULL");
    if (ms)
        for (int k = 0; k < QPM_K_COUNT; ++k) ms[k] = r->ms[k];
    if (generations) *generations = r->timed;
    if (reset) {
        for (double &v : r->ms) v = 0.0;
        r->timed = 0;
    }
    return QPM_OK;
}

QPM_API qpm_status qpm_run_load(qpm_run_handle r, const float *x, int64_t ldx)
{
    clear_error();
    QPM_REQUIRE(r != nullptr && x != nullptr, QPM_EINVAL, "run and x must not be NULL");
    QPM_REQUIRE(ldx >= r->D, QPM_EINVAL, "ldx (%lld) must be >= D (%lld)", (long long)ldx, (long long)r->D);
    const qpm_run_config &c = r->cfg;
    QPM_TRY_HIP(hipMemcpy2DAsync(r->buf[0], sizeof(float) * r->ldx, x, sizeof(float) * ldx, sizeof(float) * r->D,
                                 c.np, hipMemcpyDeviceToDevice, r->st));
    QPM_TRY_HIP(hipMemsetAsync(r->flags, 0, sizeof(uint32_t) * c.np, r->st));
    QPM_TRY_HIP(hipMemsetAsync(r->fbits, 0, sizeof(uint32_t) * 2 * ((c.np + 63) / 64), r->st));
    qpm_status st = launch_pack_pop(r->buf[0], c.np, r->D, r->ldx, r->tbits, r->ld, r->st);
    if (st == QPM_OK) st = eval_values(r);
    if (st == QPM_OK) st = launch_top3(r->f_cur, c.np, r->f64(), r->leaders, r->st);
    if (st == QPM_OK) st = launch_draws(c.np, r->D, c.seed, r->gen, c.inst, r->draws, r->st);
    if (st == QPM_OK && r->adaptive())  // F of the coming generation from the loaded population
        st = launch_adapt_F(r->f_cur, r->f64(), c.np, r->gen, c.generations, r->F_base, r->F_tab, r->st);
    return st;
}

QPM_API qpm_status qpm_run_params(qpm_run_handle r, int64_t g, float *F, float *a)
{
    clear_error();
    QPM_REQUIRE(r != nullptr, QPM_EINVAL, "run is NULL");
    QPM_REQUIRE(g >= 0 && g < r->cfg.generations, QPM_EINVAL, "generation %lld outside [0, G)", (long long)g);
    QPM_REQUIRE(!r->adaptive() || g <= r->done, QPM_EINVAL,
                "the adaptive F of generation %lld is not known yet (%lld completed)", (long long)g,
                (long long)r->done);
    float v[2] = {0.0f, 0.0f};
    QPM_TRY_HIP(hipMemcpyAsync(&v[0], r->F_tab + g, sizeof(float), hipMemcpyDeviceToHost, r->st));
    QPM_TRY_HIP(hipMemcpyAsync(&v[1], r->a_tab + g, sizeof(float), hipMemcpyDeviceToHost, r->st));
    QPM_TRY_HIP(hipStreamSynchronize(r->st));
    if (F) *F = v[0];
    if (a) *a = v[1];
    return QPM_OK;
}

QPM_API qpm_status qpm_run_read(qpm_run_handle r, float *x, int64_t ldx, void *fitness, int32_t *leaders,
                                int64_t *generation)
{
    clear_error();
    QPM_REQUIRE(r != nullptr, QPM_EINVAL, "run is NULL");
    if (x) QPM_REQUIRE(ldx >= r->D, QPM_EINVAL, "ldx (%lld) must be >= D (%lld)", (long long)ldx, (long long)r->D);
    const PopView pv = r->view();
    if (x) {
        qpm_status st = launch_gather(pv, nullptr, r->cfg.np, x, ldx, r->st);
        if (st != QPM_OK) return st;
    }
    const size_t es = r->f64() ? sizeof(double) : sizeof(float);
    if (fitness) QPM_TRY_HIP(hipMemcpyAsync(fitness, r->f_cur, es * r->cfg.np, hipMemcpyDeviceToDevice, r->st));
    if (leaders) QPM_TRY_HIP(hipMemcpyAsync(leaders, r->leaders, sizeof(int32_t) * 3, hipMemcpyDeviceToHost, r->st));
    QPM_TRY_HIP(hipStreamSynchronize(r->st));
    if (generation) *generation = r->done;
    return QPM_OK;
}

QPM_API qpm_status qpm_run_best(qpm_run_handle r, float *best_x, uint32_t *best_bits, qpm_run_stats *stats)
{
    clear_error();
    QPM_REQUIRE(r != nullptr, QPM_EINVAL, "run is NULL");
    qpm_status st = launch_top3(r->f_cur, r->cfg.np, r->f64(), r->best, r->st);
    if (st != QPM_OK) return st;
    const PopView pv = r->view();
    if (best_x) {
        if ((st = launch_gather(pv, r->best, 1, best_x, r->D, r->st)) != QPM_OK) return st;
        if (best_bits && (st = launch_pack_row(best_x, r->D, best_bits, r->st)) != QPM_OK) return st;
    } else if (best_bits) {
        float *tmp = nullptr;
        QPM_TRY_HIP(hipMallocAsync(reinterpret_cast<void **>(&tmp), sizeof(float) * r->D, r->st));
        st = launch_gather(pv, r->best, 1, tmp, r->D, r->st);
        if (st == QPM_OK) st = launch_pack_row(tmp, r->D, best_bits, r->st);
        (void)hipFreeAsync(tmp, r->st);
        if (st != QPM_OK) return st;
    }
    int32_t bi[3] = {0, 0, 0};
    QPM_TRY_HIP(hipMemcpyAsync(bi, r->best, sizeof(bi), hipMemcpyDeviceToHost, r->st));
    QPM_TRY_HIP(hipStreamSynchronize(r->st));
    if (stats) {
        double bf = 0.0;
        if (r->f64()) {
            QPM_TRY_HIP(hipMemcpy(&bf, static_cast<double *>(r->f_cur) + bi[0], sizeof(double), hipMemcpyDeviceToHost));
        } else {
            float v = 0.0f;
            QPM_TRY_HIP(hipMemcpy(&v, static_cast<float *>(r->f_cur) + bi[0], sizeof(float), hipMemcpyDeviceToHost));
            bf = v;
        }
        stats->best_fitness = bf;
        stats->best_index = bi[0];
        stats->generations = r->done;
        // evaluations per generation: trials and candidates (HWSDA), trials
        // (DE), candidates of the omega wolves (GWO)
        const int64_t np = r->cfg.np;
        const int64_t per_gen = r->cfg.algo == QPM_ALGO_DE ? np : (r->cfg.algo == QPM_ALGO_GWO ? np - 3 : 2 * np - 3);
        stats->fitness_evals = np + r->done * per_gen;
        stats->domain_evals = static_cast<double>(stats->fitness_evals) * static_cast<double>(r->D);
    }
    return QPM_OK;
}

QPM_API qpm_status qpm_run_polish(qpm_run_handle r, int32_t steps, float eta, int32_t *accepted)
{
    clear_error();
    QPM_REQUIRE(r != nullptr, QPM_EINVAL, "run is NULL");
    QPM_REQUIRE(steps >= 0 && steps <= 100000, QPM_EINVAL, "steps must be in [0, 1e5] (got %d)", (int)steps);
    QPM_REQUIRE(eta >= 0.0f && eta <= 1e6f, QPM_EINVAL, "eta must be finite and >= 0");
    QPM_REQUIRE(r->obj == nullptr, QPM_ENOTSUP, "polish relaxes |d_eff|^2, not the multi-wavelength objective");
    const qpm_run_config &c = r->cfg;
    const qpm_prec p = static_cast<qpm_prec>(c.prec);
    const int64_t ldx = r->ldx, D = r->D;
    const FitPlan pl3 = plan_fitness(*r->d, p, 3, QPM_FIT_AUTO);
    if (!r->pol) {
        hipError_t e = hipMalloc(&r->pol, sizeof(float) * 9 * ldx);
        if (e == hipSuccess) e = hipMalloc(&r->pol_S, sizeof(double) * 6);
        if (e == hipSuccess) e = hipMalloc(&r->pol_f, sizeof(float) * 6);
        if (e == hipSuccess) e = hipMalloc(&r->pol_fc, sizeof(double) * 3);
        if (e == hipSuccess) e = hipMalloc(&r->pol_bits, sizeof(uint32_t) * r->W * 64);
        if (e == hipSuccess) e = hipMalloc(&r->pol_acc, sizeof(uint32_t));
        const size_t wsb = fitness_workspace_bytes(pl3, 64);
        if (e == hipSuccess && wsb) e = hipMalloc(&r->pol_ws, wsb);
        int64_t ne = 0;
        if (e == hipSuccess && qpm_relax_edges_size(static_cast<qpm_design>(const_cast<qpm_design_s *>(
                                                        static_cast<const qpm_design_s *>(r->d))),
                                                    p, 3, &ne) != QPM_OK)
            e = hipErrorInvalidValue;
        if (e == hipSuccess) e = hipMalloc(&r->pol_edges, sizeof(double) * ne);
        if (e == hipSuccess) e = hipMemsetAsync(r->pol, 0, sizeof(float) * 9 * ldx, r->st);
        static const float ones[3] = {1.0f, 1.0f, 1.0f};
        if (e == hipSuccess) e = hipMemcpyAsync(r->pol_f + 3, ones, sizeof(ones), hipMemcpyHostToDevice, r->st);
        if (e == hipSuccess) e = hipMemsetAsync(r->pol_bits, 0, sizeof(uint32_t) * r->W * 64, r->st);
        if (e != hipSuccess) {
            set_error("polish allocation failed: %s", hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? QPM_ENOMEM : QPM_EHIP;
        }
    }
    float *theta = r->pol, *grad = r->pol + 3 * ldx, *y = r->pol + 6 * ldx;
    auto *dh = const_cast<qpm_design_s *>(static_cast<const qpm_design_s *>(r->d));
    const PopView pv = r->view();
    qpm_status st = launch_gather(pv, r->leaders, 3, theta, ldx, r->st);
    for (int32_t k = 0; k < steps && st == QPM_OK; ++k) {
        st = qpm_relax_forward(dh, p, theta, 3, ldx, r->pol_f, r->pol_S, r->pol_edges, r->st);
        if (st == QPM_OK)
            st = qpm_relax_backward(dh, p, theta, 3, ldx, r->pol_S, r->pol_edges, r->pol_f + 3, grad, ldx, r->st);
        if (st == QPM_OK) st = launch_polish_step(theta, grad, 3, D, ldx, eta, r->st);
    }
    if (st == QPM_OK) st = launch_polish_project(theta, y, 3, D, ldx, r->st);
    if (st == QPM_OK) st = launch_pack_pop(y, 3, D, ldx, r->pol_bits, 64, r->st);
    if (st == QPM_OK) st = launch_fitness(*r->d, p, r->pol_bits, 3, 64, r->pol_fc, pl3, r->pol_ws, r->st);
    if (st == QPM_OK) {
        QPM_TRY_HIP(hipMemsetAsync(r->pol_acc, 0, sizeof(uint32_t), r->st));
        st = launch_polish_accept(y, D, ldx, r->pol_fc, r->f64(), r->leaders, pv, r->f_cur, r->pol_acc, r->st);
    }
    if (st == QPM_OK && r->adaptive())  // the population entering the next generation changed
        st = launch_adapt_F(r->f_cur, r->f64(), c.np, r->gen, c.generations, r->F_base, r->F_tab, r->st);
    // a GWO run's next generation is led by the three best of the polished
    // population (a polished leader may now rank differently)
    if (st == QPM_OK && c.algo == QPM_ALGO_GWO) st = launch_top3(r->f_cur, c.np, r->f64(), r->leaders, r->st);
    if (st != QPM_OK) return st;
    uint32_t acc = 0;
    QPM_TRY_HIP(hipMemcpyAsync(&acc, r->pol_acc, sizeof(acc), hipMemcpyDeviceToHost, r->st));
    QPM_TRY_HIP(hipStreamSynchronize(r->st));
    if (accepted) *accepted = static_cast<int32_t>(acc);
    return QPM_OK;
}

QPM_API qpm_status qpm_run_destroy(qpm_run_handle r)
{
    clear_error();
    release(r);
    return QPM_OK;
}

QPM_API qpm_status qpm_run(qpm_design d, const qpm_run_config *cfg, float *best_x, uint32_t *best_bits,
                           qpm_run_stats *stats, qpm_stream s)
{
    qpm_run_handle r = nullptr;
    qpm_status st = qpm_run_create(d, cfg, s, &r);
    if (st != QPM_OK) return st;
    st = qpm_run_advance(r, cfg->generations);
    if (st == QPM_OK) st = qpm_run_best(r, best_x, best_bits, stats);
    if (st == QPM_OK) {
        // the caller's stream sees the outputs
        hipError_t e = hipStreamSynchronize(r->st);
        if (e != hipSuccess) {
            set_error("run failed: %s", hipGetErrorString(e));
            st = QPM_EHIP;
        }
    }
    release(r);
    return st;
}
