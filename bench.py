#!/usr/bin/env python3
"""Benchmark of the HWSDA hot path on one MI355X.

Workload (the fitness-throughput population): N = 10,000 domains of 2.0 um
(L = 20 mm), dk1 = 2 pi / 19.5 um^-1, dk2 = 2 pi / 6.6 um^-1, NP = 4096
genomes = 4064 iid +-1 (p = 1/2) + 32 first-order periodic seeds
(period 19.5 um, random phase). Genes carry those signs with magnitudes
uniform on (0, 1). All inputs are synthetic and seeded, resident in HBM
before timing starts.

One step = one HWSDA generation over that population, every kernel of the
hot path: DE rand/1 trials (F = 0.5, CR = 0.9), evaluation of the 4096
trials, selection, top-3 leaders, grey-wolf candidates, evaluation,
selection, generation advance -- replayed as one captured HIP graph.

value = domain evaluations per second over whole generations:
(2 NP - 3) N per generation / measured seconds. Also reported: generations/s
with FP32 and FP64 fitness and with the per-individual FP64 kernel; the
fitness kernels alone; per-kernel times from HIP events on the run's own
stream; the roofline of the dominant kernel; the CPU oracle on a bounded
sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("domain-evaluations/sec (NP×N per s) of |d_eff|^2; HWSDA generations/s vs FP64 plain")
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E, GB/s
PEAK_FP32_TFLOPS = 157.3     # vector FP32 (packed), TFLOP/s
PEAK_FP64_TFLOPS = 78.6      # vector FP64, TFLOP/s
# FP32 FMA without packed instructions (the library is built with packed
# FP32 disabled): 256 CU x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz
PEAK_FP32_NONPACKED_TFLOPS = 78.6
# LDS: 256 CU x 128 B/clk x 2.4 GHz (64-bit reads; 128-bit reads were
# measured at about twice that on this chip)
PEAK_LDS_TBS = 78.6

N_DOMAINS, NP, WIDTH = 10000, 4096, 2.0
F, CR, SEED = 0.5, 0.9, 0


def algorithmic_work(step, npop, n, lazy=True):
    """Algorithmic work of one launch of a generation step, per unit of work
    times the units one launch processes:
      gwo      8 B of HBM per gene of the np - 3 moving wolves (gene read,
               candidate written; leader rows are cache-resident) and about
               25 FP32 flops per gene;
      de       4 B of HBM per gene (target read) plus 1/8 B of trial bits,
               and 4 B more for the trial genes when every trial is stored
               (lazy = False; with accepted-only trials, the runs' choice
               at this size, the accepted genes are written after the
               selection, in the finish step); the three donor rows (12 B
               per gene) are served from the last-level cache and counted
               apart;
      fitness  10 FP32 flops per domain evaluation (np N per pass) and 6 B
               of LDS table reads per domain evaluation (one 24-byte
               triple per 4-domain block); the bit words, 1/8 B each.
    Returns a dict of {quantity: amount}."""
    genes = npop * n
    if step == "gwo":
        return {"hbm_bytes": 8.0 * (npop - 3) * n, "fp32_flops": 25.0 * (npop - 3) * n}
    if step == "de":
        return {"hbm_bytes": (4.125 if lazy else 8.125) * genes, "l2_bytes": 12.0 * genes}
    if step.startswith("fitness"):
        return {"fp32_flops": 10.0 * genes, "lds_bytes": 6.0 * genes, "hbm_bytes": genes / 8.0}
    return {}


def roofline_of(step, npop, n, seconds, f64=False):
    """The roofline entry of one step from its algorithmic work and its
    measured time per launch: the bound, achieved / peak and the fraction,
    plus the other fractions of the same work."""
    w = algorithmic_work(step, npop, n)
    if not w or seconds <= 0:
        return None
    fl_peak = PEAK_FP64_TFLOPS if f64 else PEAK_FP32_TFLOPS
    if step.startswith("fitness"):
        ach = w["fp32_flops"] / seconds / 1e12
        r = {"bound": "alu", "achieved": ach, "peak": fl_peak, "unit": "TFLOP/s", "frac": ach / fl_peak,
             "frac_of_nonpacked_fp32": ach / PEAK_FP32_NONPACKED_TFLOPS,
             "lds_tbs": w["lds_bytes"] / seconds / 1e12,
             "lds_frac": w["lds_bytes"] / seconds / 1e12 / PEAK_LDS_TBS}
    else:
        ach = w["hbm_bytes"] / seconds / 1e9
        r = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS}
        if "fp32_flops" in w:
            r["fp32_tflops"] = w["fp32_flops"] / seconds / 1e12
            r["fp32_frac_of_nonpacked"] = r["fp32_tflops"] / PEAK_FP32_NONPACKED_TFLOPS
        if "l2_bytes" in w:
            r["l2_tbs_donor_reads"] = w["l2_bytes"] / seconds / 1e12
    return r


KERNEL_SOURCES = {  # the files a kernel's code comes from (traffic records are tied to them)
    "de": ["evolve.hip", "genes.hpp", "device_common.hpp", "philox.hpp", "common.hpp"],
    "gwo": ["evolve.hip", "genes.hpp", "device_common.hpp", "philox.hpp", "common.hpp"],
    "fitness_de": ["fitness.hip", "scan.hpp", "common.hpp"],
    "fitness_gwo": ["fitness.hip", "scan.hpp", "common.hpp"],
}


def source_digest(step):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(step, []):
        with open(os.path.join(ROOT, "paper_2511_01255_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(step):
    """HBM bytes per launch from the committed counter summary of this step
    (profiles/traffic_<step>.txt: FETCH_SIZE and WRITE_SIZE scaled by a
    plain copy), or None when absent or when the kernel's sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.txt" % step)
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("source_digest") != source_digest(step):
        return None
    try:
        return float(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None



def host_cpu():
    """The host's CPU model and logical CPU count, from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as fh:
            names = [l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")]
        return "%s (%d logical CPUs)" % (names[0], len(names)) if names else None
    except OSError:
        return None


def relaxation_timing(qpm, inputs, torch, reps):
    """The relaxation workload (batch 256, N = 50,000 x 2 um, theta ~ N(0, 1)):
    forward keeping the segment edges, then the adjoint from them (the
    autograd path), reps times per precision between HIP events; ms per
    forward + adjoint, domain evaluations/s and the HBM roofline at 12 B of
    algorithmic traffic per domain (theta read by both passes, the gradient
    written)."""
    zr = inputs.uniform_boundaries(50000, 2.0)
    Dr = qpm.precompute_phases(zr, inputs.DK1, inputs.DK2)
    th = torch.from_numpy(inputs.relax_theta(256, 50000, seed=1)).cuda()
    ones = torch.ones(256, device="cuda")
    rel = {}
    for name, p_ in (("f32", qpm.PREC_F32), ("f64", qpm.PREC_F64)):
        f_, S_, E_ = qpm.relax_forward(Dr, th, p_, keep_edges=True)
        qpm.relax_backward(Dr, th, S_, ones, p_, edges=E_)
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            f_, S_, E_ = qpm.relax_forward(Dr, th, p_, keep_edges=True)
            qpm.relax_backward(Dr, th, S_, ones, p_, edges=E_)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3 / reps
        gbs = 12.0 * 256 * 50000 / t / 1e9
        rel[name] = {"ms_forward_adjoint": t * 1e3, "domain_evals_per_s": 256 * 50000 / t,
                     "hbm_gbs_at_12B_per_domain": gbs, "hbm_frac": gbs / PEAK_HBM_GBS}
    Dr.free()
    return rel


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prec", choices=["f32", "f64"], default="f32")
    ap.add_argument("--cpu-generations", type=int, default=40,
                    help="generations of the CPU oracle sample (0 = skip)")
    ap.add_argument("--no-extras", action="store_true", help="only the timed generations")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first copy a 512 MiB buffer three times (byte calibration of memory counters)")
    ap.add_argument("--relaxation-only", type=int, default=0, metavar="REPS",
                    help="time only the relaxation workload (REPS forward + adjoint per precision), print "
                         "its record as one JSON line and exit (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2511_01255_amd import inputs
    from paper_2511_01255_amd import qpm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)

    if args.calib_copy:
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.relaxation_only > 0:
        rel = relaxation_timing(qpm, inputs, torch, args.relaxation_only)
        print(json.dumps({"workload": "relaxation: batch 256 x N = 50,000 x 2.0 um, forward keeping the "
                                      "segment edges + adjoint", "relaxation": rel}), flush=True)
        return

    z = inputs.uniform_boundaries(N_DOMAINS, WIDTH)
    d = inputs.fitness_population(NP, N_DOMAINS, WIDTH, 32, seed=1)
    mag = np.random.default_rng(2).uniform(1e-3, 1.0, size=d.shape).astype(np.float32)
    genes = torch.from_numpy(np.ascontiguousarray(mag * d.astype(np.float32))).cuda()
    bits = torch.from_numpy(inputs.pack_bits(d).view(np.int32)).cuda()
    design = qpm.precompute_phases(z, inputs.DK1, inputs.DK2)
    prec = qpm.PREC_F64 if args.prec == "f64" else qpm.PREC_F32
    evals_per_gen = (2 * NP - 3) * N_DOMAINS

    def timed_run(prec_, fit_kernel, steps, warmup):
        R = qpm.Run(design, NP, warmup + steps + 32, F=F, CR=CR, seed=SEED, prec=prec_, fit_kernel=fit_kernel,
                    tune=1)
        R.load(genes)
        R.advance(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R.advance(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return R, dt

    log("[bench] main timed run: %d warmup + %d steps, prec %s" % (args.warmup, args.steps, args.prec))
    R, dt = timed_run(prec, qpm.FIT_AUTO, args.steps, args.warmup)
    value = evals_per_gen * args.steps / dt
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "domain-evaluations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {
            "workload": "fitness-throughput population: N=10000 domains x 2.0 um (L=20 mm), dk1=2pi/19.5, "
                        "dk2=2pi/6.6 um^-1, NP=4096 (4064 iid +-1 + 32 periodic seeds); one HWSDA generation "
                        "per step (DE rand/1 F=0.5 CR=0.9, GWO a: 2->0), %s fitness" % args.prec.upper(),
            "N": N_DOMAINS, "NP": NP, "generation_evals": 2 * NP - 3,
        },
        "generations_per_s": args.steps / dt,
    }

    # per-kernel times from HIP events on the run's stream
    tsteps = 20
    R.set_timing(True)
    R.timing(reset=True)
    R.advance(tsteps)
    ms, ng = R.timing()
    R.set_timing(False)
    R.destroy()
    per = {k: v / ng for k, v in ms.items()}
    out["kernel_ms"] = per
    # the dominant kernel among the steps with algorithmic work (the finish
    # steps are latency-bound one-workgroup tails and combines)
    dom = max((k for k in per if algorithmic_work(k, NP, N_DOMAINS)), key=per.get)
    roof = roofline_of(dom, NP, N_DOMAINS, per[dom] * 1e-3, f64=prec == qpm.PREC_F64)
    roof["traffic"] = measured_traffic(dom)
    roof["kernel"] = dom
    roof["kernel_ms"] = per[dom]
    out["roofline"] = roof
    out["kernel_rooflines"] = {k: roofline_of(k, NP, N_DOMAINS, v * 1e-3, f64=prec == qpm.PREC_F64)
                               for k, v in per.items() if algorithmic_work(k, NP, N_DOMAINS)}

    def guarded(name, fn):
        # an extra measurement that fails is reported and leaves the
        # headline line intact
        try:
            fn()
        except Exception as e:
            import traceback
            traceback.print_exc()
            log("[bench] %s failed: %r" % (name, e))
            out.setdefault("errors", {})[name] = repr(e)

    def _extra_fitness_kernels():
        # the same generation with each fitness kernel and precision:
        # generations/s (graph replay) and the evaluation step's kernel time
        # inside the run (HIP events around the step, eager launches)
        alt, fitk = {}, {}
        for name, p_, k_ in (("f64_table", qpm.PREC_F64, qpm.FIT_TABLE),
                             ("f64_segmented", qpm.PREC_F64, qpm.FIT_SEGMENTED),
                             ("f64_per_genome", qpm.PREC_F64, qpm.FIT_PER_GENOME),
                             ("f32_table", qpm.PREC_F32, qpm.FIT_TABLE),
                             ("f32_segmented", qpm.PREC_F32, qpm.FIT_SEGMENTED)):
            st = 40 if k_ != qpm.FIT_PER_GENOME else 10
            R2, dt2 = timed_run(p_, k_, st, 3)
            R2.set_timing(True)
            R2.advance(5)
            ms2, ng2 = R2.timing()
            R2.destroy()
            alt[name] = st / dt2
            t_fit = 0.5 * (ms2["fitness_de"] + ms2["fitness_gwo"]) / ng2 * 1e-3
            rate = NP * N_DOMAINS / t_fit
            peak = PEAK_FP64_TFLOPS if p_ == qpm.PREC_F64 else PEAK_FP32_TFLOPS
            fitk[name] = {"us_per_pass": t_fit * 1e6, "domain_evals_per_s": rate, "alg_tflops": 10 * rate / 1e12,
                          "alg_frac_of_vector_peak": 10 * rate / 1e12 / peak}
            if p_ == qpm.PREC_F32:
                fitk[name]["alg_frac_of_nonpacked_fp32_peak"] = 10 * rate / 1e12 / PEAK_FP32_NONPACKED_TFLOPS
            log("[bench] %s: %.1f generations/s, fitness pass %.1f us" % (name, st / dt2, t_fit * 1e6))
        out["generations_per_s_by_fitness"] = alt
        out["fitness_pass_in_run"] = fitk

        # the fitness entry point alone on the benchmark population: K = 200
        # back-to-back calls between HIP events on the current stream (median
        # of 5 repetitions), and one call after an idle device (median of 20)
        thr = {}
        for name, p_, k_, K_ in (("f32_table", qpm.PREC_F32, qpm.FIT_TABLE, 200),
                                 ("f64_table", qpm.PREC_F64, qpm.FIT_TABLE, 200),
                                 ("f64_per_genome", qpm.PREC_F64, qpm.FIT_PER_GENOME, 20)):
            fo = qpm.eval_fitness(design, bits, NP, p_, kernel=k_)
            reps, lat = [], []
            for _ in range(5):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(K_):
                    qpm.eval_fitness(design, bits, NP, p_, kernel=k_, out=fo)
                e1.record()
                e1.synchronize()
                reps.append(e0.elapsed_time(e1) / K_)
            for _ in range(20):
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                qpm.eval_fitness(design, bits, NP, p_, kernel=k_, out=fo)
                e1.record()
                e1.synchronize()
                lat.append(e0.elapsed_time(e1))
            t_pass = float(np.median(reps)) * 1e-3
            rate = NP * N_DOMAINS / t_pass
            thr[name] = {"passes": K_, "us_per_pass": t_pass * 1e6, "domain_evals_per_s": rate,
                         "single_call_us": float(np.median(lat)) * 1e3}
            log("[bench] fitness alone %s: %.2f us per pass, %.3g domain evaluations/s" % (name, t_pass * 1e6, rate))
        out["fitness_throughput_np4096_n10000"] = thr

    if not args.no_extras:
        guarded('fitness kernels', _extra_fitness_kernels)

    def _extra_runs():
        # full HWSDA at NP = 1024 on the same design (G = 5000 schedule,
        # seed 0, FP32 fitness): generations/s and the per-kernel split
        R3 = qpm.Run(design, 1024, 5000, F=F, CR=CR, seed=0, prec=qpm.PREC_F32, tune=1)
        R3.advance(20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R3.advance(400)
        torch.cuda.synchronize()
        t3 = (time.perf_counter() - t0) / 400
        R3.set_timing(True)
        R3.advance(20)
        ms3, ng3 = R3.timing()
        R3.destroy()
        # the whole 5000-generation run from a fresh initial population
        # (creation, tuning and initial evaluation outside the clock)
        R4 = qpm.Run(design, 1024, 5000, F=F, CR=CR, seed=0, prec=qpm.PREC_F32, tune=1)
        f_init = float(R4.read()[1].max())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R4.advance(5000)
        torch.cuda.synchronize()
        t4 = time.perf_counter() - t0
        f_end = float(R4.read()[1].max())
        R4.destroy()
        out["hwsda_np1024"] = {
            "generations_per_s": 1.0 / t3, "ms_per_generation": t3 * 1e3,
            "domain_evals_per_s": (2 * 1024 - 3) * N_DOMAINS / t3,
            "kernel_ms": {k: v / ng3 for k, v in ms3.items()},
            "full_run_5000_generations_seconds": t4,
            "best_fitness_initial_and_final": [f_init, f_end],
        }
        log("[bench] NP=1024 run: %.1f generations/s; 5000 generations in %.3f s" % (1.0 / t3, t4))

        # the same run under the paper's parameter control: F = a from 0.1 to
        # 0.01, the adaptive F (one extra one-workgroup statistics kernel per
        # generation), and the adaptive F with the discrete four-leader GWO
        ctl = {}
        for name, control, variant in (("decay", qpm.CONTROL_DECAY, 0), ("adaptive", qpm.CONTROL_ADAPTIVE, 0),
                                       ("adaptive_discrete_gwo", qpm.CONTROL_ADAPTIVE, 2)):
            Rc = qpm.Run(design, 1024, 5000, CR=CR, seed=0, prec=qpm.PREC_F32, tune=1, control=control,
                         gwo_variant=variant)
            Rc.advance(20)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Rc.advance(400)
            torch.cuda.synchronize()
            tc = (time.perf_counter() - t0) / 400
            Fs = [Rc.params(g)[0] for g in (0, 100, 420)]
            Rc.destroy()
            ctl[name] = {"generations_per_s": 1.0 / tc, "F_at_generations_0_100_420": Fs}
        out["hwsda_np1024_parameter_control"] = ctl
        log("[bench] NP=1024 parameter control: %s" % ctl)

        # batched uneven designs: 64 instances, N ~ U[1000, 50000], width
        # U[1.5, 3] um, dk1 = 2 pi / U[18, 21], dk2 = 2 pi / U[6.2, 7], NP = 256
        specs = inputs.batched_designs(64, seed=1)
        total_n = sum(len(z) - 1 for z, _, _ in specs)
        B = qpm.precompute_phases_batched([t[0] for t in specs], [t[1] for t in specs], [t[2] for t in specs])
        BR = qpm.BatchRun(B, 256, 40, F=F, CR=CR, seed=SEED, prec=prec, tune=1)
        BR.advance(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        BR.advance(10)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / 10
        BR.set_timing(True)
        BR.advance(3)
        bms, bng = BR.timing()
        BR.destroy()
        # the whole 500-generation batched run
        BR = qpm.BatchRun(B, 256, 500, F=F, CR=CR, seed=SEED, prec=prec, tune=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        BR.advance(500)
        torch.cuda.synchronize()
        tb500 = time.perf_counter() - t0
        BR.destroy()
        del B
        t_bfit = 0.5 * (bms["fitness_de"] + bms["fitness_gwo"]) / bng * 1e-3
        brate = 256 * total_n / t_bfit
        tavg = tb500 / 500
        out["batched_designs"] = {
            "instances": 64, "np": 256, "total_domains": total_n,
            # the whole 500-generation run (its average generation), and
            # generations 2-11 alone (early: most trials accepted)
            "ms_per_generation": tavg * 1e3, "generations_per_s": 1.0 / tavg,
            "domain_evals_per_s": (2 * 256 - 3) * total_n / tavg,
            "full_run_500_generations_seconds": tb500,
            "ms_per_generation_generations_2_to_11": tb * 1e3,
            "kernel_ms_generations_12_to_14": {k: v / bng for k, v in bms.items()},
            # one batched FP32 table-fitness pass: 10 algorithmic flops per
            # domain evaluation against the packed and the non-packed peak
            "fitness_pass": {"us": t_bfit * 1e6, "domain_evals_per_s": brate, "alg_tflops": 10 * brate / 1e12,
                             "alg_frac_of_vector_peak": 10 * brate / 1e12 / PEAK_FP32_TFLOPS,
                             "alg_frac_of_nonpacked_fp32_peak": 10 * brate / 1e12 / PEAK_FP32_NONPACKED_TFLOPS},
        }
        log("[bench] batched designs: %.2f ms/generation over 500 generations (%.2f early)" % (tavg * 1e3, tb * 1e3))
        out["relaxation"] = relaxation_timing(qpm, inputs, torch, 10)
        log("[bench] relaxation fwd+adjoint: %s" % out["relaxation"])

        # gradient polish of the leaders inside a run (N = 10^4, NP = 1024,
        # FP32): 20 relaxation steps every 100 generations for 500
        # generations; leaders replaced (exact +-1 fitness strictly higher)
        Rq = qpm.Run(design, 1024, 500, F=F, CR=CR, seed=0, prec=qpm.PREC_F32, tune=1)
        acc_total, t_pol = 0, 0.0
        for _ in range(5):
            Rq.advance(100)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            acc_total += Rq.polish(20, 0.05)
            t_pol += time.perf_counter() - t0
        Rq.destroy()
        out["polish_in_run"] = {"N": N_DOMAINS, "NP": 1024, "generations": 500, "polish_every": 100,
                                "steps": 20, "leaders_replaced": acc_total, "of_leaders_tried": 15,
                                "ms_per_polish": t_pol * 1e3 / 5}
        log("[bench] polish in run: %s" % out["polish_in_run"])

        # the plain FP64 HWSDA configuration: N = 256 x 2 um, NP = 32,
        # G = 200 (seed 0); the whole run on the GPU in FP64 and in FP32 (a
        # latency-bound size: one graph launch per 8 generations)
        zp = inputs.uniform_boundaries(256, 2.0)
        Dp = qpm.precompute_phases(zp, inputs.DK1, inputs.DK2)
        # (whole generations in one workgroup with the population in LDS,
        # and the multi-kernel graph path, in each precision)
        plain = {}
        for name, p_, fu in (("gpu_f64", qpm.PREC_F64, 0), ("gpu_f64_multikernel", qpm.PREC_F64, -1),
                             ("gpu_f32", qpm.PREC_F32, 0), ("gpu_f32_multikernel", qpm.PREC_F32, -1)):
            # warm-up run (first launches of the path's kernels), then the
            # timed one
            Rw = qpm.Run(Dp, 32, 200, F=F, CR=CR, seed=0, prec=p_, fused=fu)
            Rw.advance(16)
            torch.cuda.synchronize()
            Rw.destroy()
            Rp1 = qpm.Run(Dp, 32, 200, F=F, CR=CR, seed=0, prec=p_, fused=fu)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Rp1.advance(200)
            torch.cuda.synchronize()
            plain[name] = {"generations_per_s": 200 / (time.perf_counter() - t0)}
            Rp1.destroy()
        out["plain_fp64_n256_np32_g200"] = plain
        log("[bench] plain N=256 NP=32 G=200: %s" % plain)

    if not args.no_extras:
        guarded('runs and workloads', _extra_runs)

    def _extra_paper_and_objectives():
        # a run shaped like the paper's timing table (N = 6600 domains of
        # 0.1 um, L = 660 um, NP = 5000, G = 1000), with this workload's dk:
        # seconds for the whole run, next to the paper's RTX 4070 figure
        # (22.5 s, a different GPU and dk; context only)
        zp = inputs.uniform_boundaries(6600, 0.1)
        Dp = qpm.precompute_phases(zp, inputs.DK1, inputs.DK2)
        Rp = qpm.Run(Dp, 5000, 1000, F=F, CR=CR, seed=0, prec=prec, tune=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Rp.advance(1000)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        Rp.destroy()
        out["paper_shaped_run"] = {"N": 6600, "NP": 5000, "generations": 1000, "seconds": tp,
                                   "paper_rtx4070_seconds_context": 22.5}
        log("[bench] paper-shaped run (N=6600, NP=5000, G=1000): %.3f s" % tp)

        # multi-wavelength objectives on a 9 mm crystal of 3 um domains
        # (N = 3000), NP = 5000: five-wavelength SHG (dk = 2 pi / period,
        # synthetic periods) and two-wavelength coupled THG (synthetic dk
        # pairs near the workload's); a whole 1000-generation run, then the
        # per-step times of 20 generations (one objective pass = one bit
        # stream, K table walks)
        zm = inputs.uniform_boundaries(3000, 3.0)
        multi = {}
        for name, kind, dks in (("shg_5", qpm.OBJ_SHG, [(2 * np.pi / L_, 0.0) for L_ in (6.2, 6.9, 8.1, 9.3, 11.7)]),
                                ("thg_2", qpm.OBJ_THG, [(inputs.DK1, inputs.DK2), (0.30, 0.90)])):
            dsg = [qpm.precompute_phases(zm, k1, k2) for k1, k2 in dks]
            Ob = qpm.Objective(dsg, kind, 1.0, 1.0)
            npm = 5000
            Rm = qpm.Run(Ob, npm, 1020, CR=CR, seed=0, prec=qpm.PREC_F32, tune=1, control=qpm.CONTROL_DECAY)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Rm.advance(1000)
            torch.cuda.synchronize()
            tm = time.perf_counter() - t0
            # per-step HIP-event times of 20 eager generations: the objective
            # pass is the evaluation step (one partials launch over all K)
            Rm.set_timing(True)
            Rm.advance(20)
            msm, ngm = Rm.timing()
            Rm.destroy()
            ms_eval = 0.5 * (msm["fitness_de"] + msm["fitness_gwo"]) / ngm
            multi[name] = {"K": len(dks), "N": 3000, "NP": npm, "ms_per_objective_pass": ms_eval,
                           "domain_wavelength_evals_per_s": npm * 3000 * len(dks) / (ms_eval * 1e-3),
                           "run_1000_generations_seconds": tm,
                           "kernel_ms": {k: v / ngm for k, v in msm.items()}}
            del Ob, dsg
        out["multi_wavelength_objective"] = multi
        log("[bench] multi-wavelength objective: %s" % multi)

    if not args.no_extras:
        guarded('paper-shaped run and objectives', _extra_paper_and_objectives)

    def _lockstep_errors(orc):
        # the full HWSDA workload (N = 10^4, NP = 1024, G = 5000 schedule,
        # seed 0, FP32 fitness, tuned shapes, graph replay): 50 generations,
        # each replayed by the oracle from the GPU's state; a decision may go
        # the other way only on a near-tie (|f_new - f_old| within twice the
        # FP32 tolerance), counted as an adoption; rows matching no
        # admissible outcome are counted as mismatches
        npop, G, gens, tol = 1024, 5000, 50, 1e-5
        O = orc.Design(z, inputs.DK1, inputs.DK2)
        R = qpm.Run(design, npop, G, F=F, CR=CR, seed=SEED, prec=qpm.PREC_F32, tune=1)
        adopted = mismatched = 0
        for g in range(gens):
            x0 = R.read()[0].cpu().numpy()
            R.advance(1)
            xg, _, Lg, _ = R.read()
            xg = xg.cpu().numpy()
            u, _ = orc.de_step(x0, F, CR, SEED, g)
            _, fx = O.fitness(orc.sign_map(x0))
            _, fu = O.fitness(orc.sign_map(u))
            dec = fu > fx
            near = np.abs(fu - fx) <= 2 * tol * np.maximum(fu, fx)
            a = orc.a_schedule(g, G)
            outcomes = []
            for alt in (False, True):
                base = np.where((dec != alt)[:, None], u, x0)
                fb = np.where(dec != alt, fu, fx)
                base[Lg] = np.where(dec[Lg][:, None], u[Lg], x0[Lg])
                y = orc.gwo_step(base, np.array(Lg, np.int32), a, SEED, g)
                _, fy = O.fitness(orc.sign_map(y))
                acc = fy > fb
                outcomes.append((alt, base, y, acc, np.abs(fy - fb) <= 2 * tol * np.maximum(fy, fb)))
            for i in range(npop):
                found = None
                for alt, base, y, acc, ng in outcomes:
                    if alt and not near[i]:
                        continue
                    cands = [(base[i], 0)] if i in Lg else [(y[i] if acc[i] else base[i], 0),
                                                              (base[i] if acc[i] else y[i], 1)]
                    for row, flip in cands:
                        if flip and not ng[i]:
                            continue
                        if np.array_equal(row, xg[i]):
                            found = int(alt) + flip
                            break
                    if found is not None:
                        break
                if found is None:
                    mismatched += 1
                else:
                    adopted += found
        R.destroy()
        out.setdefault("errors_vs_oracle", {})["hwsda_np1024_lockstep"] = {
            "generations": gens, "decisions": gens * (2 * npop - 3), "adopted_near_ties": adopted,
            "rows_matching_no_outcome": mismatched}
        log("[bench] lockstep: %d adoptions, %d mismatches" % (adopted, mismatched))

    def _batched_errors(orc):
        # the 64 batched designs (FP32 table kernel, one launch): per
        # instance 8 first-order periodic seeds of the instance's own period
        # and 24 iid genomes; the largest plain relative error per instance
        specs = inputs.batched_designs(64, seed=1)
        npb = 32
        ldb = inputs.ld_for(npb)
        ds, rows = [], []
        for k, (zb, k1, k2) in enumerate(specs):
            nb = len(zb) - 1
            dd = np.concatenate([inputs.periodic_signs(8, nb, zb[1] - zb[0], 2 * np.pi / k1, seed=100 + k),
                                 inputs.random_signs(24, nb, seed=200 + k)])
            ds.append(dd)
            rows.append(inputs.pack_bits(dd, ldb))
        Bt = qpm.precompute_phases_batched([t[0] for t in specs], [t[1] for t in specs], [t[2] for t in specs])
        bb = torch.from_numpy(np.concatenate(rows, axis=0).view(np.int32)).cuda()
        fb = qpm.batch_eval_fitness(Bt, bb, npb, qpm.PREC_F32).double().cpu().numpy()
        per_p, per_r = [], []
        for k, (zb, k1, k2) in enumerate(specs):
            _, fo_ = orc.Design(zb, k1, k2).fitness(ds[k])
            rel = np.abs(fb[k] - fo_) / fo_
            per_p.append(float(rel[:8].max()))
            per_r.append(float(np.max(np.abs(fb[k][8:] - fo_[8:]) / np.maximum(fo_[8:], 1e-2 * np.median(fo_[8:])))))
        del Bt
        out.setdefault("errors_vs_oracle", {})["batched_64_designs_f32"] = {
            "instances": 64, "genomes_per_instance": npb,
            "periodic_max_rel_worst_instance": max(per_p), "periodic_max_rel_median_instance": float(np.median(per_p)),
            "random_max_rel_floor1pct_median_worst_instance": max(per_r)}
        log("[bench] batched errors: periodic worst %.3g" % max(per_p))

    def _oracle_timings(orc):
        # the oracle on the other run workloads, on all host threads, over a
        # few generations (each time includes the initial evaluation, so the
        # per-generation rates are slight underestimates): the full HWSDA
        # workload (N = 10^4, NP = 1024) for 20 generations and the 64
        # batched designs (NP = 256 each) for 2 generations, with the whole
        # runs (5000 and 500 generations) extrapolated from them
        res = {}
        O3 = orc.Design(z, inputs.DK1, inputs.DK2)
        t0 = time.perf_counter()
        O3.hwsda_run(1024, 20, F, CR, 0)
        t3 = time.perf_counter() - t0
        res["hwsda_np1024_n10000"] = {"generations": 20, "seconds": t3, "generations_per_s": 20 / t3,
                                      "run_5000_generations_seconds_extrapolated": 5000 * t3 / 20}
        specs = inputs.batched_designs(64, seed=1)
        t0 = time.perf_counter()
        for k, (zb, k1, k2) in enumerate(specs):
            orc.Design(zb, k1, k2).hwsda_run(256, 2, F, CR, 0, inst=k)
        t4 = time.perf_counter() - t0
        res["batched_64_designs_np256"] = {"generations": 2, "seconds": t4, "generations_per_s": 2 / t4,
                                           "run_500_generations_seconds_extrapolated": 500 * t4 / 2}
        res["threads"] = orc.num_threads()
        out.setdefault("oracle_timings", {}).update(res)
        log("[bench] oracle timings: %s" % res)

    def _relax_errors(orc):
        # the relaxation workload (batch 256, N = 5 x 10^4 x 2 um, theta ~
        # N(0, 1)): f of 8 rows against the oracle; the gradient on 64
        # sampled coordinates against the oracle's analytic gradient and its
        # central differences (h = 1e-6), normwise over the sampled rows
        Bn, nn = 256, 50000
        zr = inputs.uniform_boundaries(nn, 2.0)
        theta = inputs.relax_theta(Bn, nn, seed=5)
        Dr = qpm.precompute_phases(zr, inputs.DK1, inputs.DK2)
        Or = orc.Design(zr, inputs.DK1, inputs.DK2)
        th = torch.from_numpy(theta).cuda()
        rng = np.random.default_rng(17)
        rows = rng.integers(0, Bn, 64)
        cols = rng.integers(0, nn, 64)
        h = 1e-6
        fd = np.empty(64)
        t0 = time.perf_counter()
        for k, (b, c) in enumerate(zip(rows, cols)):
            tp = theta[b].astype(np.float64)
            tm = tp.copy()
            tp[c] += h
            tm[c] -= h
            fd[k] = np.diff(Or.relax(np.stack([tm, tp]), grad=False)[1])[0] / (2 * h)
        t_fd = time.perf_counter() - t0
        ur = np.unique(rows)
        t0 = time.perf_counter()
        _, _, go = Or.relax(theta[ur].astype(np.float64))
        t_an = time.perf_counter() - t0
        scale = float(np.max(np.abs(go)))
        an = np.array([go[np.searchsorted(ur, b), c] for b, c in zip(rows, cols)])
        fo8 = Or.relax(theta[:8].astype(np.float64), grad=False)[1]
        res = {}
        for name, p_ in (("f32", qpm.PREC_F32), ("f64", qpm.PREC_F64)):
            f_, S_ = qpm.relax_forward(Dr, th, p_)
            g_ = qpm.relax_backward(Dr, th, S_, torch.ones(Bn, device="cuda"), p_).cpu().numpy()
            got = g_[rows, cols]
            res[name] = {"f_max_rel": float(np.max(np.abs(f_[:8].double().cpu().numpy() - fo8) / fo8)),
                         "grad_normwise_vs_analytic": float(np.max(np.abs(got - an)) / scale),
                         "grad_normwise_vs_central_differences": float(np.max(np.abs(got - fd)) / scale)}
        res["oracle_analytic_vs_central_differences"] = float(np.max(np.abs(an - fd)) / scale)
        out.setdefault("errors_vs_oracle", {})["relaxation_256x50000"] = res
        out.setdefault("oracle_timings", {})["relaxation_256x50000"] = {
            "fd_set_seconds": t_fd, "fd_evaluations": 128,
            "analytic_forward_adjoint_rows": int(len(ur)), "analytic_seconds": t_an,
            "analytic_domain_evals_per_s": len(ur) * nn / t_an, "threads": orc.num_threads()}
        log("[bench] relaxation errors: %s" % res)

    def _cpu_leg():
        import oracle as orc
        # errors against the oracle, per configuration: the fitness of the
        # benchmark population (plain relative error per genome, and against
        # max(f, 1e-2 median f)), the HWSDA workload in lockstep, the batched
        # designs per instance, the relaxation's value and gradient
        Of = orc.Design(z, inputs.DK1, inputs.DK2)
        _, fo = Of.fitness(d)
        floor = 1e-2 * np.median(fo)
        errs = {}
        for name, p_, k_ in (("f32_table", qpm.PREC_F32, qpm.FIT_TABLE),
                             ("f32_segmented", qpm.PREC_F32, qpm.FIT_SEGMENTED),
                             ("f64_table", qpm.PREC_F64, qpm.FIT_TABLE),
                             ("f64_segmented", qpm.PREC_F64, qpm.FIT_SEGMENTED)):
            fg = qpm.eval_fitness(design, bits, NP, prec=p_, kernel=k_).double().cpu().numpy()
            rel = np.abs(fg - fo) / fo
            relf = np.abs(fg - fo) / np.maximum(fo, floor)
            errs[name] = {"random_max_rel": float(rel[:NP - 32].max()),
                          "random_max_rel_floor1pct_median": float(relf[:NP - 32].max()),
                          "periodic_max_rel": float(rel[NP - 32:].max())}
        out["fitness_error_vs_oracle"] = errs
        log("[bench] fitness error vs oracle: %s" % errs)
        if not args.no_extras:
            guarded("oracle timings", lambda: _oracle_timings(orc))
            guarded("lockstep errors", lambda: _lockstep_errors(orc))
            guarded("batched errors", lambda: _batched_errors(orc))
            guarded("relaxation errors", lambda: _relax_errors(orc))
        log("[bench] CPU oracle: %d generations" % args.cpu_generations)
        O = orc.Design(z, inputs.DK1, inputs.DK2)
        x = (mag * d.astype(np.float32)).astype(np.float32)
        t0 = time.perf_counter()
        _, f = O.fitness(orc.sign_map(x))
        G = args.cpu_generations
        for g in range(G):
            u, _ = orc.de_step(x, F, CR, SEED, g)
            _, fu = O.fitness(orc.sign_map(u))
            acc = fu > f
            x[acc] = u[acc]
            f[acc] = fu[acc]
            L = orc.top3(f)
            y = orc.gwo_step(x, L, orc.a_schedule(g, G), SEED, g)
            _, fy = O.fitness(orc.sign_map(y))
            acc = fy > f
            acc[L] = False
            x[acc] = y[acc]
            f[acc] = fy[acc]
        tc = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": evals_per_gen * G / tc,
            "unit": "domain-evaluations/s",
            "cores": orc.num_threads(),
            "kind": "oracle",
            "sample": "%d HWSDA generations of the same workload (plus the initial evaluation) with the "
                      "long-double CPU oracle, %.1f s" % (G, tc),
            "host_cpu": host_cpu(),
        }
        if not args.no_extras:
            # the oracle on the plain FP64 configuration (N = 256, NP = 32,
            # G = 200), beside the GPU runs of it above
            Op = orc.Design(inputs.uniform_boundaries(256, 2.0), inputs.DK1, inputs.DK2)
            t0 = time.perf_counter()
            Op.hwsda_run(32, 200, F, CR, 0)
            out["oracle_plain_fp64_n256_np32_g200"] = {
                "generations_per_s": 200 / (time.perf_counter() - t0), "cores": orc.num_threads()}
            # one fitness pass of the benchmark population on the oracle, on
            # all host threads and on one (median of 3 each; the plain run
            # above on one thread too)
            dsign = orc.sign_map(mag * d.astype(np.float32))
            one = {}
            for nt in (orc.num_threads(), 1):
                orc.set_num_threads(nt)
                ts = []
                for _ in range(3):
                    t0 = time.perf_counter()
                    O.fitness(dsign)
                    ts.append(time.perf_counter() - t0)
                one[nt] = NP * N_DOMAINS / float(np.median(ts))
            t0 = time.perf_counter()
            Op.hwsda_run(32, 200, F, CR, 0)
            plain1 = 200 / (time.perf_counter() - t0)
            orc.set_num_threads(max(one))
            out["oracle_fitness_pass_np4096_n10000"] = {
                "domain_evals_per_s_all_threads": one[max(one)], "threads": max(one),
                "domain_evals_per_s_one_thread": one[1]}
            out["oracle_plain_fp64_n256_np32_g200"]["generations_per_s_one_thread"] = plain1

    if args.cpu_generations > 0:
        guarded('cpu leg', _cpu_leg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
