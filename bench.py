"""Benchmark: cluster updates/s and time-to-1e-4 gap/site on one MI355X.

Default workload: the batched sweep of 512 periodic L x L transverse-field Ising lattices
(L ~ U{8..64}, h ~ U[0.5, 4], seed 4; 2 x 2 plaquette clusters 16 x 16 over their bonds and
sites: 3.33 M clusters, 6.66 M messages, real symmetric), entropy-smoothed Algorithm 2 with FP32
iterations replayed from captured HIP graphs in autotuned launch shapes, FP64 certification
(lambda_min of every cluster + rounding margin).  A "step" is 50 accelerated iterations
followed by one certification (extrapolation, assembly, Gibbs states, partial traces, message
updates and the dual value over the whole batch, then the certified bound); `value` is the
cluster-update rate over the timed steps.  The timed steps run at the final beta of the gap
schedule, continuing from the schedule's lower-beta stages (an untimed pre-phase), i.e. in
the regime that takes most of a solve.  The same steps in the plain FP64 form (one launch per
phase, no graph) are reported beside it, then the time to a certified gap of 1e-4 per site in
every instance for both forms, from zero messages, against per-instance references (see
plaquette_reference), and the FP64 CPU oracle on one host core and on all of them over a
bounded sample.  Inputs are synthetic, built on the host and resident in HBM before any timing
starts.

Other workloads (--workload): c2 (32 x 32 Heisenberg), c1, c3k<k>, c3t<k>, c4t, c5, ex2, ex3.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

ITERS_PER_STEP = 50
TOTAL_ITERS = 5000
BETA0, BETA_MAX = 1.0, 1024.0
Q_REF = -6144.0            # closed form: -3 J per bond, 2048 bonds (singlet on every bond)
HBM_PEAK_GBS = 8000.0
# HBM-side bytes per launch of the dominant kernel, per workload: rocprofv3 FETCH_SIZE + WRITE_SIZE
# of the kernel, each scaled by what the counter reads for a 64 MiB device copy in the same run,
# stored with the hash of the library sources (kernel_sources_hash) the counters were taken with;
# reported as null once the sources change.
TRAFFIC_BYTES = {
    # k_cluster_expm<float,false,16>, beta = 12288 (profiles/k_cluster_expm_c4_plaquette_sweep_counters.md)
    "c4": ("08381585aefdc54d", 336836217),
    # k_cluster_expm_wg<float,true,256>, beta = 64 (profiles/k_cluster_expm_wg_c3_interval_k8_counters.md)
    "c3k8": ("08381585aefdc54d", 474942516323),
    # k_cluster_pair<float,false,GIBBS> (profiles/k_cluster_pair_heisenberg32x32_traffic.md)
    "c2": ("08381585aefdc54d", 1038195),
}


def traffic_bytes(workload):
    rec = TRAFFIC_BYTES.get(workload)
    return rec[1] if rec and rec[0] == kernel_sources_hash() else None


FP32_VALU_PEAK_TFLOPS = 157.3


def schedule_iter(schedule):
    """Yield (stage index, beta) for every global iteration."""
    for s, (beta, K) in enumerate(schedule):
        for _ in range(K):
            yield s, beta


class Solver:
    """Drives Algorithm 2 stage by stage through the library, in steps of 50 iterations."""

    def __init__(self, P, f32, fused, schedule):
        self.P, self.f32, self.fused, self.schedule = P, f32, fused, schedule
        self.nu = P.zeros(f32)
        self.ze = P.zeros(f32)
        self.stage = 0
        self.state = P.new_nesterov_state(schedule[0][0])
        self.left = schedule[0][1]

    def run(self, n):
        while n > 0:
            if self.left == 0:
                self.stage += 1
                beta, K = self.schedule[self.stage]
                self.state = self.P.new_nesterov_state(beta)
                self.left = K
            m = min(n, self.left)
            self.P.step_nesterov(self.nu, self.ze, self.state, m, fused=self.fused)
            self.left -= m
            n -= m


def timed_solve(P, f32, fused, steps, warmup, schedule, torch):
    """Warm up on a throwaway state, then time `steps` steps from nu = 0."""
    if warmup > 0:
        w = Solver(P, f32, fused, schedule)
        for _ in range(warmup):
            w.run(ITERS_PER_STEP)
            P.certify(w.nu)
        torch.cuda.synchronize()
    S = Solver(P, f32, fused, schedule)
    q = torch.zeros((steps, P.n_inst), dtype=torch.float64, device="cuda")
    mg = torch.zeros_like(q)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    from paper_2609_40336_amd import lrh
    for k in range(steps):
        S.run(ITERS_PER_STEP)
        lrh.lrh_certify(P.h, S.nu, lrh.LRH_F32 if f32 else 0, q[k], mg[k])
        ev[k + 1].record()
    torch.cuda.synchronize()
    t_total = ev[0].elapsed_time(ev[-1]) / 1e3
    t_at = [ev[0].elapsed_time(ev[k + 1]) / 1e3 for k in range(steps)]
    bound = (q - mg)[:, 0].cpu().numpy()
    n_sites = P.desc.n_sites
    gaps = (Q_REF - bound) / n_sites
    tte = None
    for k in range(steps):
        if gaps[k] <= 1e-4:
            tte = t_at[k]
            break
    return dict(seconds=t_total, iters=steps * ITERS_PER_STEP, bound=float(bound[-1]),
                gap_per_site=float(gaps[-1]), time_to_1e4=tte, nu=S.nu)


def kernel_timing(P, torch, f32=True, reps=20):
    """Average duration of one fused iteration (one k_cluster_pair launch plus 1/64 of the
    chunk's parameter upload and closing message update), timed with HIP events on the
    stream the graph is launched on."""
    S = Solver(P, f32, True, [(BETA0, 10 ** 9)])
    S.run(64)  # capture
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        S.run(64)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / (reps * 64)


def algorithmic_work(P):
    """Algorithmic work per iteration, fixed before measuring: bytes B = w (6 sum_msg s_f + 2 sum_{f
    with parents} s_f) with s the packed size, w = 4 (FP32); flops F = 11 D^3 per real
    cluster (symmetric eigen-decomposition with vectors plus the U diag U^T rebuild)."""
    w = 4
    s_msg = 0
    for b in P.buckets:
        s_msg += b["M"] * b["comps"]
    with_parents = set(int(c) for c in P.msg_child)
    s_par = 0
    for c in with_parents:
        D = 2 ** len(P.clusters[c])
        s_par += D * (D + 1) // 2 if P.is_real else D * D
    B = w * (6 * s_msg + 2 * s_par)
    F = 0
    for c in P.clusters:
        D = 2 ** len(c)
        F += (11 if P.is_real else 44) * D ** 3
    return B, F


def kernel_sources_hash():
    """First 16 hex digits of the sha256 over every kernel and host source of the library."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2609_40336_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(desc, budget_s=15.0):
    """The FP64 oracle, untuned, on one core: Algorithm 2 iterations of the same workload
    until the time budget is spent (at least 2)."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    from oracle import lrh_oracle as O
    ctx = threadpool_limits(1) if threadpool_limits else None
    try:
        R = O.Relaxation(desc)
        nu = R.zeros()
        ze = R.copy(nu)
        beta = BETA0
        L = R.lipschitz(beta)
        th = 1.0
        n = 0
        t0 = time.perf_counter()
        while True:
            eta = R.axpby(1.0 - th, nu, th, ze)
            _, g = R.grad_beta(eta, beta)
            ze = R.symmetrise({k: ze[k] + g[k] / (th * L) for k in ze})
            nu = R.symmetrise(R.axpby(1.0 - th, nu, th, ze))
            th = O.theta_next(th)
            n += 1
            if n >= 2 and time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    return dict(value=R.n_clusters * n / dt, unit="cluster updates/s", cores=1, kind="oracle",
                sample=f"{n} Algorithm 2 iterations of the 32x32 Heisenberg workload (FP64 NumPy, "
                       f"one thread), {dt:.1f} s")


FP64_MFMA_PEAK_TFLOPS = 78.6
FP64_VALU_PEAK_TFLOPS = 78.6


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def message_kernel_roofline(P, nu, ze, beta, torch, reps=3):
    """HBM roofline of the accelerated message update (a6): every message component costs six
    accesses of the state precision (read nu, zeta, T and R; write nu and zeta); the launches
    of every message bucket are timed live with HIP events, on scratch copies of the state."""
    nu2, ze2 = nu.clone(), ze.clone()
    us = P.time_messages(nu2, ze2, beta, reps)
    del nu2, ze2
    w = 4 if nu.dtype == torch.float32 else 8
    nbytes = sum(b["M"] * b["comps"] * 6 * w for b in P.buckets)
    sec = sum(us) / 1e6
    gbs = nbytes / sec / 1e9
    return dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=gbs / HBM_PEAK_GBS,
                kernel="k_msg (accelerated message update, one launch per message bucket)",
                per_iteration=dict(bytes=nbytes, seconds=sec), buckets_us=[round(u, 3) for u in us])


def dominant_kernel_roofline(P, nus, beta, f32, torch, reps=3):
    """Roofline of the slowest cluster-kernel launch of one pass: the bucket's algorithmic flops
    (11 D^3 real / 44 D^3 complex per cluster: symmetric QR with vectors plus the
    reconstruction) over its launch duration, timed live with HIP events on the launch stream
    at each message state in `nus` (the start and end of the timed region) and averaged.  The
    scaling-and-squaring kernel (shape 0) runs in FP64 on the matrix cores, the others on the
    vector ALUs in the iteration precision."""
    per_state = [P.time_buckets(nu, beta, reps) for nu in nus]
    us = [float(np.mean(col)) for col in zip(*per_state)]
    shapes = P.shapes()
    b = int(np.argmax(us))
    sh = shapes[b]
    D, n = sh["De"], sh["n"]
    F = (11 if P.is_real else 44) * D ** 3 * n
    t = us[b] * 1e-6
    W = sh["W"] if f32 else sh.get("W", 0)
    if W in (0, 4) and D >= 16 and beta > 0:
        bound, peak = "mfma", FP64_MFMA_PEAK_TFLOPS
        kind = ("scaling-and-squaring Gibbs kernel (matrix cores: FP64 polynomial and first four squarings, "
                "FP32 for the rest; priced against the FP64 peak)" if (f32 and W == 0) else
                "scaling-and-squaring Gibbs kernel (FP64 MFMA)")
    else:
        bound = "alu"
        peak = FP32_VALU_PEAK_TFLOPS if f32 else FP64_VALU_PEAK_TFLOPS
        kind = "Jacobi cluster kernel (vector ALU)"
    ach = F / t / 1e12
    extra = {}
    if bound == "mfma":
        from paper_2609_40336_amd import lrh
        sus = lrh.lrh_measure_fp64_mfma(0)
        extra = dict(sustained_fp64_mfma_tflops=sus, frac_of_sustained=ach / sus,
                     executed_tflops_note="the exponential executes (4 + s) products of 2 D^3 flops per "
                                          "cluster with float messages, (5 + s) with double ones, s the "
                                          "squarings (more than the 11 D^3 counted here)")
    return dict(bound=bound, achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak, traffic=None, **extra,
                kernel=f"{kind}, bucket D={D} (n={n}), beta={beta:g}",
                per_launch=dict(flops=F, seconds=t,
                                seconds_per_state=[round(x[b] * 1e-6, 7) for x in per_state]),
                all_buckets_us=[round(u, 3) for u in us])


# CPU sample of the interval chains: long enough that the mix of cluster sizes, which sets the
# cost per cluster update, is within about 3 % of the 4096-site chain's (the top level dominates)
C3_CPU_SITES = 128


def c3_mix(n, k):
    """Clusters per top cluster of the interval hierarchy Y_k on an n-site chain (levels 1..k,
    n - m + 1 intervals of m sites at level m)."""
    return sum(n - m + 1 for m in range(1, k + 1)) / (n - k + 1)


def oracle_rate(desc, budget_s, beta=1.0):
    """The FP64 oracle, untuned, on one core: Algorithm 2 iterations at fixed beta until the
    budget is spent (at least 2).  Returns (cluster updates/s, iterations, seconds)."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    from oracle import lrh_oracle as O
    ctx = threadpool_limits(1) if threadpool_limits else None
    try:
        R = O.Relaxation(desc)
        nu = R.zeros()
        ze = R.copy(nu)
        L = R.lipschitz(beta)
        th = 1.0
        n = 0
        t0 = time.perf_counter()
        while True:
            eta = R.axpby(1.0 - th, nu, th, ze)
            _, g = R.grad_beta(eta, beta)
            ze = R.symmetrise({k: ze[k] + g[k] / (th * L) for k in ze})
            nu = R.symmetrise(R.axpby(1.0 - th, nu, th, ze))
            th = O.theta_next(th)
            n += 1
            if n >= 2 and time.perf_counter() - t0 > budget_s:
                break
        dt = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    return R.n_clusters * n / dt, n, dt


def _line(metric_value, args, name, P, extra):
    out = {
        "metric": "cluster updates/s", "value": metric_value, "unit": "cluster updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "data": "synthetic",
        "config": {"workload": name, "clusters": P.n_clusters, "messages": P.n_msgs, "instances": P.n_inst},
    }
    out.update(extra)
    return out


def long_reference(P, n_sites, torch, stages=19, per=6000):
    """Per-instance reference for the time to a certified gap where no closed form or symmetry
    reduction exists: the best certified value per site of a long FP64 run (beta = 2^0 .. 2^18,
    `per` accelerated iterations per stage: 114 000 by default, at least ten times the solves it
    serves), and the improvement of its last stage per site."""
    nu, ze = P.zeros(False), P.zeros(False)
    best = np.full(P.n_inst, -np.inf)
    last = float("inf")
    for s_ in range(stages):
        st = P.new_nesterov_state(2.0 ** s_)
        P.step_nesterov(nu, ze, st, per, fused=True)
        q, mg, _ = P.certify(nu)
        b = (q - mg).cpu().numpy() / n_sites
        if s_:
            last = float(np.max(b - best))
        best = np.maximum(best, b)
    return best, last, stages * per


def time_to_gap(P, desc, n_sites, torch, target=1e-4):
    """Time to a certified gap of `target` per site in every instance, fused FP32 and plain FP64,
    on the gap schedule (gap_stages, solve_to_gap) against long_reference."""
    t0 = time.perf_counter()
    ref, last, its = long_reference(P, n_sites, torch)
    print(f"[bench] reference: {its} FP64 iterations in {time.perf_counter() - t0:.1f} s, last stage moved "
          f"{last:.1e} per site", file=sys.stderr, flush=True)
    out = {"target_gap_per_site": target,
           "schedule": f"beta = 2^s for {GAP_STAGE_ITERS} iterations each (Algorithm 2 restarted per stage) "
                       f"while below {GAP_BETA_FINAL:g}, then beta = {GAP_BETA_FINAL:g} without restarts; "
                       f"FP64 certification every {GAP_CHECK} iterations, inside the timing",
           "reference": f"best certified value per site of an FP64 run of {its} iterations (beta = 2^0 .. 2^18)",
           "reference_last_stage_improvement_per_site": last}
    for key, f32, fused in (("fused_fp32", True, True), ("plain_fp64", False, False)):
        r, _, _ = solve_to_gap(P, f32, fused, ref, n_sites, torch)
        out[key] = r
        if r["iterations"] is not None and 10 * r["iterations"] > its:
            out[key]["reference_shorter_than_10x"] = True
    print(f"[bench] time to {target:g} gap/site: {out}", file=sys.stderr, flush=True)
    return out


# ---- time to a certified gap (default workload) ----------------------------------------------
GAP_TARGET = 1e-4          # certified gap per site, every instance
GAP_STAGE_ITERS = 500      # iterations per beta stage while beta doubles (each stage restarts)
GAP_BETA_FINAL = 12288.0   # final inverse temperature, held without restarts until the target
GAP_CHECK = 250            # certification cadence (its cost is inside the measured time)
GAP_MAX_ITERS = 60000


def gap_stages(beta_final=GAP_BETA_FINAL, K=GAP_STAGE_ITERS):
    """beta = 2^s for K iterations each while below beta_final, then beta_final (open-ended)."""
    betas = []
    b = 1.0
    while b < beta_final:
        betas.append(b)
        b *= 2.0
    return [(bb, K) for bb in betas] + [(beta_final, None)]


def plaquette_reference(hs, torch, L=3, stages=21, per=3000):
    """Relaxation optimum per site of a periodic TFIM plaquette lattice for every field h.

    A periodic lattice is translation invariant; Q is concave, so averaging an optimal message
    set over the translations gives a translation-invariant optimal one, and with invariant
    messages every plaquette, bond and site repeats the same three augmented Hamiltonians: the
    optimum per site is the same for every L >= 3 (the poset is locally the same).  It is taken
    as the best certified value per site of a 3 x 3 lattice per field, solved in FP64 with
    beta = 2^0 .. 2^20 and `per` accelerated iterations per stage.  Returns (values per site,
    improvement of the last stage per site), the latter bounding how far the reference still
    is from converged."""
    import lrh_workloads as W
    from paper_2609_40336_amd import lrh
    d = W.tfim_plaquette_batch([L] * len(hs), hs, name="plaquette_reference")
    P = lrh.Problem(d, 0)
    nu, ze = P.zeros(), P.zeros()
    best = np.full(len(hs), -np.inf)
    last = 0.0
    for st_ in range(stages):
        st = P.new_nesterov_state(2.0 ** st_)
        P.step_nesterov(nu, ze, st, per, fused=True)
        q, mg, _ = P.certify(nu)
        b = (q - mg).cpu().numpy() / (L * L)
        last = float(np.max(b - best)) if st_ else float("inf")
        best = np.maximum(best, b)
    P.close()
    return best, last


class _ScaledSteps:
    """A problem whose accelerated states use L = beta Lambda_G / (2 f) (see solve_to_gap)."""

    def __init__(self, P, f):
        self._P, self._f = P, f

    def __getattr__(self, name):
        return getattr(self._P, name)

    def new_nesterov_state(self, beta):
        return self._P.new_nesterov_state(beta, beta * self._P.Lambda / (2.0 * self._f))


def solve_to_gap(P, f32, fused, ref, n_sites, torch, max_iters=GAP_MAX_ITERS, step_scale=1.0):
    """Algorithm 2 on the gap schedule from nu = 0, certified every GAP_CHECK iterations, until
    every instance is within GAP_TARGET per site of its reference (or max_iters).  Timed with
    HIP events around the whole solve, certifications and their read-back included.
    step_scale > 1 divides the step constant L = beta Lambda_G / 2 (an upper bound of the
    gradient's Lipschitz constant) by it: a heuristic outside the method's guarantee, for the
    --step-scale measurement only."""
    from paper_2609_40336_amd import lrh
    stages = gap_stages()
    if step_scale != 1.0:
        P = _ScaledSteps(P, step_scale)
    nu, ze = P.zeros(f32), P.zeros(f32)
    q = torch.zeros(P.n_inst, dtype=torch.float64, device="cuda")
    mg = torch.zeros_like(q)
    e0, e1 = _events(torch)
    torch.cuda.synchronize()
    e0.record()
    k, si = 0, 0
    st = P.new_nesterov_state(stages[0][0])
    left = stages[0][1]
    reached, gap, trace = None, None, []
    while k < max_iters:
        n = GAP_CHECK if left is None else min(GAP_CHECK, left)
        P.step_nesterov(nu, ze, st, n, fused=fused)
        k += n
        lrh.lrh_certify(P.h, nu, lrh.LRH_F32 if f32 else 0, q, mg)
        gaps = ref - (q - mg).cpu().numpy() / n_sites    # synchronises
        gap = float(np.max(gaps))
        if k % 2500 == 0:
            trace.append((k, gap))
            print(f"[bench]   {'fp32 fused' if fused else 'fp64 plain'}: {k} iterations, max gap "
                  f"{gap:.3g} per site", file=sys.stderr, flush=True)
        if gap <= GAP_TARGET:
            reached = k
            break
        if left is not None:
            left -= n
            if left == 0:
                si += 1
                st = P.new_nesterov_state(stages[si][0])
                left = stages[si][1]
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    return dict(seconds=sec if reached else None, iterations=reached, iterations_run=k,
                max_gap_per_site_at_end=gap, solve_seconds=sec,
                cluster_updates_per_s_whole_solve=P.n_clusters * k / sec,
                max_gap_every_2500_iterations=[(kk, float("%.3g" % g)) for kk, g in trace]), nu, ze


def _oracle_worker(job):
    """One CPU process: Algorithm 2 iterations (FP64 oracle, one BLAS thread) at fixed beta on the
    plaquette lattices `job` = (Ls, hs, beta, budget); returns (cluster updates, seconds)."""
    Ls, hs, beta, budget = job
    from threadpoolctl import threadpool_limits
    import lrh_workloads as W
    from oracle import lrh_oracle as O
    with threadpool_limits(1):
        R = O.Relaxation(W.tfim_plaquette_batch(Ls, hs, name="cpu_sample"))
        nu = R.zeros()
        ze = R.copy(nu)
        L = R.lipschitz(beta)
        th, n = 1.0, 0
        t0 = time.perf_counter()
        while True:
            eta = R.axpby(1.0 - th, nu, th, ze)
            _, g = R.grad_beta(eta, beta)
            ze = R.symmetrise({k: ze[k] + g[k] / (th * L) for k in ze})
            nu = R.symmetrise(R.axpby(1.0 - th, nu, th, ze))
            th = O.theta_next(th)
            n += 1
            if n >= 2 and time.perf_counter() - t0 > budget:
                break
        return R.n_clusters * n, time.perf_counter() - t0


def cpu_oracle_legs(Ls, hs, beta, budget):
    """The untuned FP64 oracle on the host: one process on one instance of the sweep, then one
    process per host core (at most 16, the host share of one GPU), each on its own instance, all
    for `budget` seconds.  Runs in fresh processes before this process touches the GPU."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    ncpu = os.cpu_count() or 1
    ncores = max(1, min(ncpu, 16))
    out = {}
    with ctx.Pool(1) as pool:
        u, dt = pool.map(_oracle_worker, [([Ls[0]], [hs[0]], beta, budget)])[0]
    out["one_core"] = dict(value=u / dt, unit="cluster updates/s", cores=1, kind="oracle",
                           sample=f"Algorithm 2 iterations at beta = {beta:g} on instance 0 of the sweep "
                                  f"(L = {Ls[0]}, h = {hs[0]:.3f}; FP64 NumPy, one thread), {dt:.1f} s")
    jobs = [([Ls[i % len(Ls)]], [hs[i % len(hs)]], beta, budget) for i in range(ncores)]
    t0 = time.perf_counter()
    with ctx.Pool(ncores) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    upd = sum(u for u, _ in res)
    span = max(dt for _, dt in res)
    out["all_cores"] = dict(value=upd / span, unit="cluster updates/s", cores=ncores, kind="oracle",
                            os_cpu_count=ncpu,
                            sample=f"{ncores} processes, one instance of the sweep each (instances 0..{ncores - 1}, "
                                   f"L = {sorted(set(int(Ls[i % len(Ls)]) for i in range(ncores)))}), Algorithm 2 "
                                   f"iterations at beta = {beta:g} (FP64 NumPy, one thread each), {span:.1f} s "
                                   f"({wall:.1f} s wall with start-up)")
    return out


def profile_traffic_run(P, torch, beta, passes=3):
    """Short run for hardware counters: `passes` Gibbs passes over every cluster bucket (FP32
    messages, seeded noise of scale 0.3) at `beta` and one FP64 certification of the same
    messages, then a 64 MiB device copy (a plain copy kernel of known size, to scale FETCH_SIZE /
    WRITE_SIZE)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    nu = (0.3 * torch.randn(P.nu_len, generator=g, device="cuda", dtype=torch.float64)).float()
    for _ in range(passes):
        P.dual_eval(nu, beta, grad=True)
    P.certify(nu)
    src = torch.ones(16 * 2 ** 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile_traffic": "done", "beta": beta, "passes": passes, "copy_bytes": src.numel() * 4}))


def bench_c4_default(args, torch, cpu):
    """The default line: the 512-lattice plaquette sweep (see the module docstring)."""
    import lrh_workloads as W
    from paper_2609_40336_amd import lrh
    t0 = time.perf_counter()
    desc = W.workload_c4()
    hs = np.asarray(desc.meta["hs"], dtype=np.float64)
    n_sites = np.bincount(desc.site_instance, minlength=desc.n_instances).astype(np.float64)
    P = lrh.Problem(desc, 0)
    print(f"[bench] {desc.name}: {P.n_clusters} clusters, {P.n_msgs} messages, built in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    cache = os.path.join(os.environ.get("TMPDIR", "/tmp"), "lrh_shapes.json")
    shapes = P.autotune(True, cache)
    P.autotune(False, cache)
    beta = GAP_BETA_FINAL
    ips = ITERS_PER_STEP
    if args.profile_traffic:
        return profile_traffic_run(P, torch, beta)

    # Pre-phase (untimed): the gap schedule's stages below the final beta (beta = 1, 2, ..., 8192,
    # GAP_STAGE_ITERS iterations each, FP32 fused), so that the timed steps run in the regime that
    # takes most of a solve: beta = beta_final near the optimum, where the scaling-and-squaring
    # kernel's squaring count no longer changes.
    t1 = time.perf_counter()
    pre_nu, pre_ze = P.zeros(True), P.zeros(True)
    pre_iters = 0
    for b, K in gap_stages()[:-1]:
        P.step_nesterov(pre_nu, pre_ze, P.new_nesterov_state(b), K, fused=True)
        pre_iters += K
    torch.cuda.synchronize()
    print(f"[bench] pre-phase: {pre_iters} iterations at beta = 1 .. {gap_stages()[-2][0]:g} in "
          f"{time.perf_counter() - t1:.1f} s", file=sys.stderr, flush=True)

    def timed_steps(f32, fused, steps, warmup):
        """`warmup` untimed steps, then `steps` timed steps (ips iterations + one FP64
        certification each) of Algorithm 2 at the final beta, continuing from the pre-phase's
        messages (widened to FP64 for the FP64 form) with a fresh accelerated state, as the
        solve's final stage does.  A short spin kernel marks each end of the timed region in a
        kernel trace.  Returns the seconds and the messages at the start and end of the timed
        region."""
        nu, ze = P.zeros(f32), P.zeros(f32)
        nu.copy_(pre_nu)
        ze.copy_(pre_ze)
        st = P.new_nesterov_state(beta)
        for _ in range(warmup):
            P.step_nesterov(nu, ze, st, ips, fused=fused)
            P.certify(nu)
        nu_start = nu.clone()
        q = torch.zeros((steps, P.n_inst), dtype=torch.float64, device="cuda")
        mg = torch.zeros_like(q)
        e0, e1 = _events(torch)
        torch.cuda.synchronize()
        torch.cuda._sleep(1000)
        e0.record()
        for k in range(steps):
            P.step_nesterov(nu, ze, st, ips, fused=fused)
            lrh.lrh_certify(P.h, nu, lrh.LRH_F32 if f32 else 0, q[k], mg[k])
        e1.record()
        torch.cuda._sleep(1000)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3, nu_start, nu, ze

    iters = args.steps * ips
    sec, nu_a, nu, ze = timed_steps(True, True, args.steps, args.warmup)
    print(f"[bench] fused fp32: {sec:.3f} s for {iters} iterations at beta = {beta:g}", file=sys.stderr, flush=True)
    roof = dominant_kernel_roofline(P, [nu_a, nu], beta, True, torch)
    roof["traffic"] = traffic_bytes("c4")
    roof64 = dominant_kernel_roofline(P, [nu], 64.0, True, torch)
    msg_roof = message_kernel_roofline(P, nu, ze, beta, torch)
    del nu, ze, nu_a
    sec_plain, _, _, _ = timed_steps(False, False, args.steps, min(args.warmup, 1))
    del pre_nu, pre_ze
    print(f"[bench] plain fp64: {sec_plain:.3f} s for {iters} iterations", file=sys.stderr, flush=True)
    tte = tte_plain = None
    ref_last = None
    if not args.no_gap:
        t1 = time.perf_counter()
        ref, ref_last = plaquette_reference(hs, torch)
        print(f"[bench] per-field references in {time.perf_counter() - t1:.1f} s (last stage moved "
              f"{ref_last:.1e} per site)", file=sys.stderr, flush=True)
        tte, nu, ze = solve_to_gap(P, True, True, ref, n_sites, torch, step_scale=args.step_scale)
        del nu, ze
        print(f"[bench] fused fp32 to {GAP_TARGET:g}: {tte}", file=sys.stderr, flush=True)
        if not args.no_plain_gap:
            tte_plain, nu, ze = solve_to_gap(P, False, False, ref, n_sites, torch, step_scale=args.step_scale)
            del nu, ze
            print(f"[bench] plain fp64 to {GAP_TARGET:g}: {tte_plain}", file=sys.stderr, flush=True)
    nchk, nnf = P.check()
    out = {
        "metric": "cluster updates/s and time-to-1e-4 gap/site: fused vs plain FP64, 1 MI355X",
        "value": P.n_clusters * iters / sec, "unit": "cluster updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 iterations, f64 certify", "data": "synthetic",
        "config": {"workload": "tfim_plaquette_sweep_512_L8to64_h0.5to4_seed4_plaquettes_nesterov",
                   "instances": P.n_inst, "clusters": P.n_clusters, "messages": P.n_msgs,
                   "iters_per_step": ips, "beta_of_timed_steps": beta,
                   "timed_steps_start": f"after the gap schedule's {pre_iters} iterations below beta = {beta:g} "
                                        f"and {args.warmup} warm-up steps at it",
                   "parallelism": "single_gpu"},
        "us_per_iteration": sec / iters * 1e6,
        "time_to_1e-4_gap_per_site_s": tte["seconds"] if tte else None,
        "time_to_gap": {
            "fused_fp32": tte, "plain_fp64": tte_plain,
            "target_gap_per_site": GAP_TARGET,
            "schedule": f"beta = 2^s for {GAP_STAGE_ITERS} iterations each (Algorithm 2 restarted per stage) "
                        f"while below {GAP_BETA_FINAL:g}, then beta = {GAP_BETA_FINAL:g} without restarts; "
                        f"FP64 certification every {GAP_CHECK} iterations, inside the timing",
            "reference": "per field h: best certified value per site of the 3 x 3 periodic lattice "
                         "(translation invariance), FP64, beta up to 2^20",
            "reference_last_stage_improvement_per_site": ref_last,
            "step_constant": "L = beta Lambda_G / 2" if args.step_scale == 1.0 else
                             f"L = beta Lambda_G / (2 x {args.step_scale:g}) (heuristic, --step-scale)",
        },
        "plain_fp64": {"value": P.n_clusters * iters / sec_plain, "unit": "cluster updates/s",
                       "form": "FP64, one launch per phase and message bucket, no graph, the same batch",
                       "time_to_1e-4_gap_per_site_s": tte_plain["seconds"] if tte_plain else None},
        "shapes": shapes, "jacobi_noconv": nchk, "nonfinite": nnf,
        "roofline": roof, "roofline_at_beta_64": roof64, "roofline_message_kernel": msg_roof,
    }
    if cpu:
        out["cpu_baseline"] = cpu["all_cores"]
        out["cpu_baseline_one_core"] = cpu["one_core"]
    print(json.dumps(out))


def bench_rate(workload, args, torch):
    """Batched Algorithm 2 on a large workload: FP32 iterations replayed from captured graphs
    with autotuned launch shapes, beta doubling 1 -> 1024 over 11 stages of
    --iters-per-stage iterations, FP64 certification after every stage; then the same
    schedule in the plain FP64 form (one launch per phase, no graph).  There is no closed-form
    optimum for these workloads: for the plaquette sweep and the intervals k <= 5 the time to a
    1e-4 gap per site in every instance is measured as well (time_to_gap)."""
    import lrh_workloads as W
    from paper_2609_40336_amd import lrh
    t0 = time.perf_counter()
    reference = False
    if workload == "c4rate":
        reference = False   # the default line measures the sweep's time to the gap
        desc = W.workload_c4()
        sample = W.workload_c4(n_inst=2)
        name = "tfim_plaquette_sweep_512_L8to64_h0.5to4_nesterov_fp32"
        sample_txt = "a 2-instance plaquette sweep drawn the same way"
        ips = 50
    elif workload == "c4t":
        reference = False
        desc = W.workload_c4(two_level=True)
        sample = W.workload_c4(n_inst=2, two_level=True)
        name = "tfim_plaquette_sweep_512_L8to64_h0.5to4_two_level_nesterov_fp32"
        sample_txt = "a 2-instance plaquette sweep drawn the same way, two-level family"
        ips = 50
    elif workload.startswith("c3k"):
        k = int(workload[3:])
        desc = W.workload_c3(k)
        reference = k <= 5
        sample = W.interval_chain_gue(C3_CPU_SITES, k, 0.1, seed=3)
        name = f"interval_chain_gue_n4096_eps0.1_Y{k}_nesterov_fp32"
        sample_txt = (f"the same interval hierarchy Y{k} on a {C3_CPU_SITES}-site chain "
                      f"({c3_mix(C3_CPU_SITES, k):.2f} clusters per top cluster; {c3_mix(4096, k):.2f} on the full chain)")
        ips = 10 if k >= 8 else 50
    elif workload.startswith("c3t"):
        k = int(workload[3:])
        desc = W.workload_c3(k, two_level=True)
        reference = k <= 5
        sample = W.interval_chain_gue(C3_CPU_SITES, k, 0.1, seed=3, two_level=True)
        name = f"interval_chain_gue_n4096_eps0.1_two_level_windows{k}_nesterov_fp32"
        sample_txt = (f"the same two-level family (windows of {k} and their overlaps) on a "
                      f"{C3_CPU_SITES}-site chain")
        ips = 10 if k >= 8 else 50
    else:
        raise SystemExit(f"unknown workload {workload}")
    if args.iters_per_stage:
        ips = args.iters_per_stage
    P = lrh.Problem(desc, 0)
    t_build = time.perf_counter() - t0
    print(f"[bench] {desc.name}: {P.n_clusters} clusters, {P.n_msgs} messages, built in {t_build:.1f} s",
          file=sys.stderr, flush=True)
    cache = os.path.join(os.environ.get("TMPDIR", "/tmp"), "lrh_shapes.json")
    shapes = P.autotune(True, cache)
    P.autotune(False, cache)
    print(f"[bench] shapes {shapes}", file=sys.stderr, flush=True)
    if args.profile_traffic:
        return profile_traffic_run(P, torch, 64.0, passes=2)
    sched = [(2.0 ** s, ips) for s in range(11)]

    def timed_schedule(f32, fused):
        for _ in range(args.warmup):
            Solver(P, f32, fused, sched).run(ips)
        torch.cuda.synchronize()
        S = Solver(P, f32, fused, sched)
        q = torch.zeros((len(sched), P.n_inst), dtype=torch.float64, device="cuda")
        mg = torch.zeros_like(q)
        ev = [_events(torch)[0] for _ in range(len(sched) + 1)]
        torch.cuda.synchronize()
        ev[0].record()
        for k in range(len(sched)):
            S.run(ips)
            lrh.lrh_certify(P.h, S.nu, lrh.LRH_F32 if f32 else 0, q[k], mg[k])
            ev[k + 1].record()
        torch.cuda.synchronize()
        sec = ev[0].elapsed_time(ev[-1]) / 1e3
        stage_ms = [ev[k].elapsed_time(ev[k + 1]) / ips for k in range(len(sched))]
        t_at = [ev[0].elapsed_time(ev[k + 1]) / 1e3 for k in range(len(sched))]
        return S, sec, stage_ms, (q - mg).cpu().numpy(), t_at

    iters = len(sched) * ips
    S, sec, stage_ms, bounds, t_at = timed_schedule(True, True)
    bound = bounds[-1]
    print(f"[bench] fused fp32: {sec:.3f} s for {iters} iterations", file=sys.stderr, flush=True)
    nchk, nnf = P.check()
    n_sites = np.bincount(desc.site_instance, minlength=desc.n_instances)
    roof = dominant_kernel_roofline(P, [S.nu], 64.0, True, torch)
    roof["traffic"] = traffic_bytes(workload)
    msg_roof = message_kernel_roofline(P, S.nu, S.ze, 64.0, torch)
    del S
    _, sec_plain, stage_plain, bounds_plain, t_at_plain = timed_schedule(False, False)
    bound_plain = bounds_plain[-1]
    print(f"[bench] plain fp64: {sec_plain:.3f} s for {iters} iterations", file=sys.stderr, flush=True)
    tte = time_to_gap(P, desc, n_sites, torch) if (reference and args.time_to_gap) else None
    children = {c for (_, c) in P.message_keys()}
    n_top = sum(1 for c in P.clusters if c not in children)
    extra = {
        "ms_per_step": sec / len(sched) * 1e3, "dtype": "f32 iterations, f64 certify",
        "us_per_iteration": sec / iters * 1e6,
        "top_cluster_updates_per_s": n_top * iters / sec,
        "schedule": f"beta = 2^s, s = 0..10, {ips} iterations per stage, FP64 certify after each stage",
        "ms_per_iteration_by_stage": [round(x, 4) for x in stage_ms],
        "mean_certified_bound_per_site": float(np.mean(bound / n_sites)),
        "time_to_1e-4_gap_per_site_s": tte,
        "plain_fp64": {"value": P.n_clusters * iters / sec_plain, "unit": "cluster updates/s",
                       "ms_per_iteration_by_stage": [round(x, 4) for x in stage_plain],
                       "mean_certified_bound_per_site": float(np.mean(bound_plain / n_sites))},
        "shapes": shapes, "jacobi_noconv": nchk, "nonfinite": nnf, "roofline": roof,
        "roofline_message_kernel": msg_roof,
    }
    if not args.no_cpu:
        v, n, dt = oracle_rate(sample, args.cpu_budget)
        extra["cpu_baseline"] = dict(value=v, unit="cluster updates/s", cores=1, kind="oracle",
                                     sample=f"{n} Algorithm 2 iterations (beta = 1) of {sample_txt} "
                                            f"(FP64 NumPy, one thread), {dt:.1f} s")
    out = _line(P.n_clusters * iters / sec, args, name, P, extra)
    out["config"]["iters_per_stage"] = ips
    print(json.dumps(out))


E0_TFIM16 = -16.146050955496804   # open TFIM chain n = 16, J = 1, h = 0.5 (free-fermion closed form)


def bench_c1(args, torch):
    """Algorithm 1 on the open TFIM chain n = 16 (complex storage, FP64): 2000 subgradient
    iterations with alpha_k = 1/sqrt(k+1), one launch per phase; best certified bound and the
    bracket against the exact ground energy."""
    import lrh_workloads as W
    from paper_2609_40336_amd import lrh
    desc = W.workload_c1()
    P = lrh.Problem(desc, 0)
    K = 2000

    def run(n):
        nu, nb = P.zeros(), P.zeros()
        qb = torch.full((P.n_inst,), -math.inf, dtype=torch.float64, device="cuda")
        P.step_subgrad(nu, nb, qb, 0, n)
        return nu, nb, qb
    for _ in range(args.warmup):
        run(50)
    torch.cuda.synchronize()
    e0, e1 = _events(torch)
    e0.record()
    nu, nb, qb = run(K)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    b, mg, _ = P.certify(nb)
    torch.cuda.synchronize()
    cert = float((b - mg).item())
    nchk, nnf = P.check()
    B = 16 * (3 * sum(bk["M"] * bk["comps"] for bk in P.buckets))
    t_it = sec / K
    extra = {
        "ms_per_step": sec * 1e3, "dtype": "complex f64", "us_per_iteration": t_it * 1e6,
        "q_best": float(qb.item()), "certified_bound": cert, "exact_E0": E0_TFIM16, "anderson_bound": -23.0,
        "bracket_ok": bool(-23.0 - 1e-9 <= cert <= E0_TFIM16 + 1e-9),
        "jacobi_noconv": nchk, "nonfinite": nnf,
        "roofline": dict(bound="hbm", achieved=B / t_it / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                         frac=B / t_it / 1e9 / HBM_PEAK_GBS, traffic=None,
                         kernel="one Algorithm 1 iteration (cluster kernels + reduce + message update)",
                         per_launch=dict(bytes=B, seconds=t_it)),
    }
    if not args.no_cpu:
        from oracle import lrh_oracle as O
        R = O.Relaxation(desc)
        t0 = time.perf_counter()
        n = 0
        while True:
            n += 50
            O.subgradient(R, n)
            if time.perf_counter() - t0 > args.cpu_budget / 2:
                break
        dt = time.perf_counter() - t0
        tot = sum(range(50, n + 1, 50))
        extra["cpu_baseline"] = dict(value=R.n_clusters * tot / dt, unit="cluster updates/s", cores=1, kind="oracle",
                                     sample=f"{tot} Algorithm 1 iterations on the same chain (FP64 NumPy, one "
                                            f"thread), {dt:.1f} s")
    out = _line(P.n_clusters * K / sec, args, "tfim_open_chain_n16_h0.5_level1_subgradient_2000it_fp64", P, extra)
    out["steps"] = 1
    print(json.dumps(out))


def bench_c5(args, torch):
    """Forward and adjoint on the 64x64 triangular XXZ lattice (FP64, beta = 4): T = 16
    accelerated steps plus the certified value, then the reverse pass giving the gradient of
    that value with respect to all 12288 couplings."""
    import lrh_workloads as W
    from paper_2609_40336_amd import lrh
    desc = W.workload_c5()
    P = lrh.Problem(desc, 0)
    beta, T = 4.0, 16
    L = beta * P.Lambda / 2.0

    def forward():
        nu, ze = P.zeros(), P.zeros()
        st = P.new_nesterov_state(beta, L=L)
        P.step_nesterov(nu, ze, st, T, fused=False)
        b, mg, _ = P.certify(nu)
        return nu, b
    for _ in range(max(args.warmup, 1)):
        forward()
        P.unrolled_bound_grad(beta, T, L)
    torch.cuda.synchronize()
    reps = 5
    e0, e1 = _events(torch)
    e0.record()
    for _ in range(reps):
        nu, b = forward()
    e1.record()
    torch.cuda.synchronize()
    t_fwd = e0.elapsed_time(e1) / 1e3 / reps
    e0.record()
    for _ in range(reps):
        bb, pb, _ = P.unrolled_bound_grad(beta, T, L)
    e1.record()
    torch.cuda.synchronize()
    t_grad = e0.elapsed_time(e1) / 1e3 / reps
    roof = dominant_kernel_roofline(P, [nu], beta, False, torch)
    nchk, nnf = P.check()
    extra = {
        "ms_per_step": t_fwd * 1e3, "dtype": "f64", "beta": beta, "T": T,
        "forward_s": t_fwd, "value_and_gradient_s": t_grad, "adjoint_cost_ratio": t_grad / t_fwd,
        "bound": float(bb.item()), "grad_abs_mean": float(pb.abs().mean().item()),
        "jacobi_noconv": nchk, "nonfinite": nnf, "roofline": roof,
    }
    if not args.no_cpu:
        from oracle import lrh_oracle as O
        R = O.Relaxation(desc)
        t0 = time.perf_counter()
        O.unrolled_bound_grad(R, beta, 2, L=R.lipschitz(beta))
        dt = time.perf_counter() - t0
        extra["cpu_baseline"] = dict(value=R.n_clusters * 2 * 2 / dt, unit="cluster updates/s", cores=1,
                                     kind="oracle",
                                     sample=f"value and gradient after T = 2 steps on the full lattice (oracle "
                                            f"reverse mode, FP64 NumPy, one thread; forward + reverse counted as 2 "
                                            f"updates per cluster and step), {dt:.1f} s")
    out = _line(P.n_clusters * T / t_fwd, args, "xxz_triangular_64x64_delta0.5_beta4_T16_value_and_gradient_fp64",
                P, extra)
    out["steps"] = reps
    print(json.dumps(out))


EX3_EPS = [0.02, 0.0139, 0.00965, 0.0067, 0.00465, 0.00323, 0.00224, 0.002]


def bench_ex3(args, torch):
    """Iterations to epsilon (the paper's comparison of the subgradient and smooth methods):
    level-1 relaxation of 16-site open chains (Heisenberg J = 1 with an on-site X field 0.5,
    anisotropic Heisenberg (2, -3, 0.5) with the same field, critical TFIM J = h = 1, a seeded
    random chain).

    * Algorithm 1 with the constant step alpha = eps / (2 Delta_G) (Sec. 4.1.1): since the ground
      projector is scale-invariant, it is Algorithm 1 with step 1 on H / alpha.
    * Algorithm 2 at the fixed beta = 2 Gamma / (n eps) of the smoothing-error lemma: it is
      Algorithm 2 at beta = 1 on beta H, with nu rescaled by beta.
    So every (model, eps) pair is one instance of a single batched problem per method.
    Convergence: certified Q(nu^k) within eps per site of the relaxation optimum, taken as the
    best certified value of a long beta-continuation run (beta up to 2^16) and of every run
    here.  Exponent p: least-squares fit of log(iterations) against log(1 / eps)."""
    import lrh_workloads as W
    from paper_2609_40336_amd import lrh
    n = 16
    models = {
        "heisenberg_field0.5": W.heisenberg_chain(n, field_x=0.5),
        "xyz_2_-3_0.5_field0.5": W.anisotropic_heisenberg_chain(n, field_x=0.5),
        "tfim_critical": W.tfim_chain(n, 1.0, 1.0, complex_storage=False),
        "random": W.random_chain(n, seed=7),
    }
    names = list(models)
    descs = [models[k] for k in names]
    Delta, d = 2, 2
    Gamma = (n - 1) * math.log(4.0) + n * math.log(2.0)
    t0 = time.perf_counter()
    # relaxation optimum: long accelerated run with beta continuation, certified
    Pr = lrh.Problem(W.batch_scaled(descs, [1.0] * len(descs), "ex3_ref"), 0)
    Sr = Solver(Pr, False, True, [(2.0 ** s, 800) for s in range(17)])
    qref = np.full(len(names), -np.inf)
    for _ in range(17):
        Sr.run(800)
        b, mg, _ = Pr.certify(Sr.nu)
        qref = np.maximum(qref, (b - mg).cpu().numpy())
    print(f"[ex3] reference optimum per site {qref / n}", file=sys.stderr, flush=True)
    out_models = {k: {} for k in names}
    # ---- Algorithm 1 ----
    inst = [(m, e) for m in range(len(names)) for e in EX3_EPS]
    alphas = [e / (2.0 * Delta) for (_, e) in inst]
    P1 = lrh.Problem(W.batch_scaled([descs[m] for (m, _) in inst], [1.0 / a for a in alphas], "ex3_sub"), 0)
    nu, nb = P1.zeros(), P1.zeros()
    qb = torch.full((P1.n_inst,), -math.inf, dtype=torch.float64, device="cuda")
    chunk, kmax = 20000, int(args.ex3_max_iters)
    first = [None] * len(inst)
    qbest = np.full(len(inst), -np.inf)
    k0 = 0
    while k0 < kmax and any(f is None for f in first):
        qh = torch.empty((chunk, P1.n_inst), dtype=torch.float64, device="cuda")
        P1.step_subgrad(nu, nb, qb, k0, chunk, step_kind=1, step_scale=1.0, q_hist=qh)
        q = qh.cpu().numpy() * np.asarray(alphas)[None, :]
        qbest = np.maximum(qbest, q.max(axis=0))
        for i, (m, e) in enumerate(inst):
            if first[i] is None:
                hit = np.nonzero((qref[m] - q[:, i]) / n <= e)[0]
                if len(hit):
                    first[i] = k0 + int(hit[0]) + 1
        k0 += chunk
    # ---- Algorithm 2 ----
    betas = [2.0 * Gamma / (n * e) for (_, e) in inst]
    P2 = lrh.Problem(W.batch_scaled([descs[m] for (m, _) in inst], betas, "ex3_smooth"), 0)
    nu2, ze2 = P2.zeros(), P2.zeros()
    st = P2.new_nesterov_state(1.0)
    check, kmax2 = 5, int(args.ex3_max_iters) // 4
    first2 = [None] * len(inst)
    qbest2 = np.full(len(inst), -np.inf)
    k = 0
    while k < kmax2 and any(f is None for f in first2):
        P2.step_nesterov(nu2, ze2, st, check, fused=True)
        k += check
        b, mg, _ = P2.certify(nu2)
        q = (b - mg).cpu().numpy() / np.asarray(betas)
        qbest2 = np.maximum(qbest2, q)
        for i, (m, e) in enumerate(inst):
            if first2[i] is None and (qref[m] - q[i]) / n <= e:
                first2[i] = k
    torch.cuda.synchronize()
    # runs that ended above the long run's value raise the reference (it is a lower bound)
    for i, (m, e) in enumerate(inst):
        qref[m] = max(qref[m], qbest[i], qbest2[i])
    secs = time.perf_counter() - t0

    def fit(eps, its):
        pts = [(e, t) for e, t in zip(eps, its) if t is not None]
        if len(pts) < 3 or len(set(t for _, t in pts)) == 1:
            return None, None   # too few points, or no dependence on eps (optimum at the start)
        x = np.log([1.0 / e for e, _ in pts])
        y = np.log([float(t) for _, t in pts])
        p, c = np.polyfit(x, y, 1)
        r2 = 1.0 - np.sum((y - (p * x + c)) ** 2) / max(np.sum((y - y.mean()) ** 2), 1e-300)
        return float(p), float(r2)
    for m, key in enumerate(names):
        idx = [i for i, (mm, _) in enumerate(inst) if mm == m]
        eps = [inst[i][1] for i in idx]
        its1 = [first[i] for i in idx]
        its2 = [first2[i] for i in idx]
        p1, r1 = fit(eps, its1)
        p2, r2 = fit(eps, its2)
        out_models[key] = {
            "relaxation_optimum_per_site": float(qref[m] / n),
            "optimal_at_start": bool(all(t == 1 for t in its1)),
            "subgradient": {"iterations": its1, "exponent": p1, "r2": r1},
            "smooth": {"iterations": its2, "exponent": p2, "r2": r2, "checked_every": check},
        }
    out = {
        "metric": "iterations to eps per site (subgradient vs smooth), exponent of 1/eps",
        "experiment": "eps-scaling of Algorithms 1 and 2 on 16-site chains, level-1 relaxation",
        "eps": EX3_EPS, "models": out_models, "n_gpus": 1, "seconds": secs, "data": "synthetic",
        "max_iterations": {"subgradient": int(args.ex3_max_iters), "smooth": kmax2},
        "paper_context": {"subgradient_exponent": "<= 2 (random), 1.33-1.8 (others)",
                          "smooth_exponent": "0.8 (random), about 0.5 (others)"},
    }
    print(json.dumps(out))


def bench_ex2(args, torch):
    """Size dependence of the optimal multiplier norm (the assumption behind both rate
    theorems): mean Frobenius norm of the messages nu_{e->f} at the end of a long accelerated
    run (beta = 2^s, s = 0..12, 400 iterations per stage, FP64) on open chains of N sites,
    N = 8 .. 256, for the isotropic Heisenberg, anisotropic Heisenberg (2, -3, 0.5), critical
    TFIM and seeded random chains.  All (model, N) pairs run as one batched problem; the
    certified bound per site is reported beside the norm, and the fitted slope of norm
    against N measures any size dependence."""
    import lrh_workloads as W
    from paper_2609_40336_amd import lrh
    Ns = [8, 16, 32, 64, 128, 256]
    makers = {
        "heisenberg": lambda N: W.heisenberg_chain(N),
        "xyz_2_-3_0.5": lambda N: W.anisotropic_heisenberg_chain(N),
        "tfim_critical": lambda N: W.tfim_chain(N, 1.0, 1.0, complex_storage=False),
        "random": lambda N: W.random_chain(N, seed=11),
    }
    inst = [(k, N) for k in makers for N in Ns]
    desc = W.batch_scaled([makers[k](N) for (k, N) in inst], [1.0] * len(inst), "ex2")
    t0 = time.perf_counter()
    P = lrh.Problem(desc, 0)
    S = Solver(P, False, True, [(2.0 ** s, 400) for s in range(13)])
    S.run(13 * 400)
    b, mg, _ = P.certify(S.nu)
    torch.cuda.synchronize()
    bound = (b - mg).cpu().numpy()
    secs = time.perf_counter() - t0
    norms = [[] for _ in inst]
    for (par, ch), m in P.to_dense(S.nu).items():
        norms[int(desc.site_instance[ch[0]])].append(float(np.linalg.norm(m)))
    out_models = {}
    for k in makers:
        idx = [i for i, (kk, _) in enumerate(inst) if kk == k]
        mean = [float(np.mean(norms[i])) for i in idx]
        slope = float(np.polyfit(np.asarray(Ns, float), np.asarray(mean), 1)[0])
        out_models[k] = {"N": Ns, "mean_message_norm": mean, "slope_per_site": slope,
                         "certified_bound_per_site": [float(bound[i] / inst[i][1]) for i in idx]}
    out = {"metric": "mean optimal message Frobenius norm vs chain length",
           "experiment": "size independence of the optimal multipliers, level-1 relaxation of open chains",
           "models": out_models, "iterations": 13 * 400, "seconds": secs, "n_gpus": 1, "data": "synthetic",
           "paper_context": "no visible correlation of the average optimal multiplier norm with N"}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0,
                    help="timed steps (default 20 on c4, 100 = the whole 5000-iteration solve on c2)")
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-plain-gap", action="store_true",
                    help="default workload: skip the plain FP64 solve to the gap target")
    ap.add_argument("--no-gap", action="store_true",
                    help="default workload: timed steps and rooflines only, no solves to the gap target "
                         "(the command of the kernel-trace profiles)")
    ap.add_argument("--workload", default="c4",
                    help="c4 (default: the 512-lattice plaquette sweep, rate and time to 1e-4), c2 (the "
                         "32x32 Heisenberg solve), c1 (TFIM chain, Algorithm 1), c3k<k> "
                         "(interval hierarchy Y_k on the n = 4096 GUE chain), c3t<k> (the same chain with the "
                         "two-level family: windows of k sites and their overlaps), c4rate (the sweep on the "
                         "older beta 1 -> 1024 schedule; c4t: the two-level family of plaquettes and shared bonds), "
                         "c5 (64x64 XXZ value and coupling gradient), ex3 (iterations-to-eps experiment), "
                         "ex2 (optimal message norm vs chain length)")
    ap.add_argument("--step-scale", type=float, default=1.0,
                    help="default line: divide the accelerated step constant L = beta Lambda_G / 2 of the "
                         "time-to-gap solves by this factor (a heuristic outside the method's guarantee; "
                         "the line records it)")
    ap.add_argument("--time-to-gap", action="store_true",
                    help="c3k2..c3k5, c3t2..c3t5: also measure the time to a 1e-4 certified gap per site "
                         "(the default c4 line always does)")
    ap.add_argument("--ex3-max-iters", type=float, default=4e5,
                    help="ex3: iteration cap of Algorithm 1 (Algorithm 2: a quarter of it)")
    ap.add_argument("--iters-per-stage", type=int, default=0,
                    help="c3k<k>, c3t<k>, c4: iterations per beta stage (default 50; 10 for k = 8)")
    ap.add_argument("--profile-traffic", action="store_true",
                    help="short run for hardware counters, then a 64 MiB device copy (a plain copy kernel "
                         "of known size, for calibration): c2 4 fused graph chunks; c4, c3k<k>, c3t<k>: Gibbs "
                         "passes over every bucket (c4 at beta 12288, the others at 64)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the path is single-GPU; --gpus {args.gpus} "
              f"is not supported)", file=sys.stderr)
        sys.exit(2)
    if args.steps <= 0:
        args.steps = 20 if args.workload == "c4" else TOTAL_ITERS // ITERS_PER_STEP
    if args.workload == "c4":
        # CPU legs first, in fresh processes, before this process touches the GPU
        cpu = None
        if not args.no_cpu:
            import lrh_workloads as W
            sweep = W.workload_c4()
            Ls, hs = list(sweep.meta["Ls"]), list(sweep.meta["hs"])
            del sweep
            cpu = cpu_oracle_legs(Ls, hs, GAP_BETA_FINAL, args.cpu_budget)
            print(f"[bench] cpu oracle: {cpu}", file=sys.stderr, flush=True)
        import torch
        return bench_c4_default(args, torch, cpu)
    import torch
    import lrh_workloads as W
    from paper_2609_40336_amd import lrh

    if args.workload != "c2":
        args.steps = 1
        if args.workload == "c1":
            return bench_c1(args, torch)
        if args.workload == "c5":
            return bench_c5(args, torch)
        if args.workload == "ex3":
            return bench_ex3(args, torch)
        if args.workload == "ex2":
            return bench_ex2(args, torch)
        return bench_rate(args.workload, args, torch)
    desc = W.workload_c2(32)
    P = lrh.Problem(desc, 0)
    schedule = lrh.nesterov_schedule(BETA0, BETA_MAX, TOTAL_ITERS)
    if args.profile_traffic:
        S = Solver(P, True, True, [(BETA0, 10 ** 9)])
        for _ in range(4):
            S.run(64)
        src = torch.ones(16 * 2 ** 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_traffic": "done", "copy_bytes": src.numel() * 4}))
        return
    print(f"[bench] workload {desc.name}: {P.n_clusters} clusters, {P.n_msgs} messages", file=sys.stderr,
          flush=True)
    fused = timed_solve(P, True, True, args.steps, args.warmup, schedule, torch)
    print(f"[bench] fused fp32: {fused['seconds']:.4f} s for {fused['iters']} iterations", file=sys.stderr,
          flush=True)
    plain = timed_solve(P, False, False, args.plain_steps, 1, schedule, torch)
    print(f"[bench] plain fp64: {plain['seconds']:.4f} s for {plain['iters']} iterations", file=sys.stderr,
          flush=True)
    t_it = kernel_timing(P, torch)
    nchk, nnf = P.check()
    B, F = algorithmic_work(P)
    t_B, t_F = B / (HBM_PEAK_GBS * 1e9), F / (FP32_VALU_PEAK_TFLOPS * 1e12)
    if t_B >= t_F:
        roof = dict(bound="hbm", achieved=B / t_it / 1e9, peak=HBM_PEAK_GBS, unit="GB/s")
    else:
        roof = dict(bound="alu", achieved=F / t_it / 1e12, peak=FP32_VALU_PEAK_TFLOPS, unit="TFLOP/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = traffic_bytes("c2")
    roof["kernel"] = "k_cluster_pair<float,false,MODE_GIBBS> (one fused iteration)"
    roof["per_launch"] = dict(bytes=B, flops=F, seconds=t_it)
    updates = P.n_clusters * fused["iters"]
    out = {
        "metric": "cluster updates/s and time-to-1e-4 gap/site: fused vs plain FP64, 1 MI355X",
        "value": updates / fused["seconds"],
        "unit": "cluster updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fused["seconds"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 iterations, f64 certify",
        "data": "synthetic",
        "config": {"workload": "heisenberg_af_32x32_periodic_level1_nesterov_beta1to1024_5000it",
                   "clusters": P.n_clusters, "messages": P.n_msgs,
                   "iters_per_step": ITERS_PER_STEP, "parallelism": "single_gpu"},
        "time_to_1e-4_gap_per_site_s": fused["time_to_1e4"],
        "certified_bound": fused["bound"],
        "gap_per_site": fused["gap_per_site"],
        "plain_fp64": {"value": P.n_clusters * plain["iters"] / plain["seconds"], "unit": "cluster updates/s",
                       "steps": args.plain_steps, "time_to_1e-4_gap_per_site_s": plain["time_to_1e4"],
                       "gap_per_site": plain["gap_per_site"]},
        "jacobi_noconv": nchk, "nonfinite": nnf,
        "roofline": roof,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(desc, args.cpu_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
