#!/usr/bin/env python3
"""Throughput of the projected-product hot path on one MI355X.

Default workload: the batched form, 64 independent instances of uneven sizes
(n1, n2, n4 uniform in [64, 512], n3 in [32, 256], p in [4, 32], float32
N(0,1) data, a random orthonormal Q each, k = p/2).  One step is one replay
of the captured graph that computes, for every instance, C = A *_Q B
(Def. 3.1) and the rank-k truncated tSVDQ of A (Alg. 4.1 steps 2-3).  The
same line carries what the metric compares the batched and the compensated
forms with: the same 64 instances as sequential unbatched float32 calls, the
hyperspectral-shaped tSVDQ (512 x 512 x 224 bfloat16, p = 32, k = 16) in the
float32 and split-bfloat16 (x3) transforms, the differentiation-shaped
product in float32, bf16x3 and plain bf16, and the relative errors of every
timed result against the float64 oracle (plain bf16's as reported numbers).

Prints ONE JSON line (metric, value in GFLOP/s of the nominal flop count,
roofline of the dominant kernel measured with HIP events on the launch stream,
and the float64 CPU oracle timed on this host as a baseline).  Per-kernel
details go to stderr, and as JSON to the file named by --details.

    python bench.py [--steps K] [--warmup W] [--workload batched|video|hyper|...]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_MFMA_PEAK = 157.3         # TFLOP/s dense
BF16_MFMA_PEAK = 2500.0        # TFLOP/s dense
FP64_MFMA_PEAK = 78.6          # TFLOP/s dense

# HBM bytes per launch of the dominant kernel, from rocprofv3 --pmc FETCH_SIZE
# and WRITE_SIZE runs of the same workload, scaled by the plain-copy
# calibration (2.0 x FETCH_SIZE + 1.0 x WRITE_SIZE, KiB -> bytes); keyed by
# (workload, precision mode, kernel).  Absent means not measured for the
# kernel as it is now.
TRAFFIC_BYTES = {
    ("video", "default", "jacobi_gram_f32"): 9930752,     # 2 x 2587.3 + 4523.4 KiB
    ("hat-video", "bf16x3", "hat"): 67830000,              # 2 x 30120 + 6000 KiB
    ("hat-hyper", "bf16x3", "hat"): 151400000,             # 2 x 57560 + 32768 KiB
    ("hat-video", "default", "hat"): 67827698,             # 2 x 30119 + 6000 KiB
}

METRIC = "\u22c6_Q/tSVDQ GFLOP/s + % roofline, BF16-comp & batched vs FP32 at rel err\u22641e-5"


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info()
                    if d.get("user_api") == "blas"] or [1])
    except Exception:  # threadpoolctl missing
        return os.cpu_count()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batched",
                    choices=["video", "hyper", "diff", "tiny", "copy", "hat-video", "hat-hyper",
                             "proj-video", "qprod", "batched", "svdii-video", "u3-video",
                             "u3-video-f64", "tsvdq-backward-video", "facewise"])
    ap.add_argument("--count", type=int, default=64, help="instances of the batched workload")
    ap.add_argument("--prec", default="default")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall-clock budget of the CPU-oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--details", default=None, help="file for the per-kernel details (JSON)")
    ap.add_argument("--no-compare", action="store_true",
                    help="batched workload: skip the float32/compensated comparisons and oracle errors")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# workloads: each returns (step_fn, flops_per_step, info dict, kernel models)
# kernel model: name -> (bound, units_per_launch_fn) giving algorithmic
# bytes ("hbm") or flops ("mfma": float32 matrix cores, "mfma64": float64)
# per launch
# ---------------------------------------------------------------------------

def svd_nominal_flops(n1, n2, p):
    """Golub-Van Loan R-SVD count for Sigma, U1, V of an m x n matrix
    (m >= n): 6 m n^2 + 20 n^3, per face."""
    mx, mn = max(n1, n2), min(n1, n2)
    return p * (6.0 * mx * mn * mn + 20.0 * mn ** 3)


JACOBI_KERNELS = ("jacobi_gram_f32", "jacobi_gram_f64", "jacobi_block_f32", "jacobi_block_f64",
                  "jacobi_global_f32", "jacobi_global_f64")


def jacobi_models(svd_flops):
    """Roofline models of the Jacobi sweep kernels: the nominal SVD work of a
    step spread evenly over that step's sweep launches (float32 coarse and
    float64 polishing sweeps), so each phase carries the share of its own
    launches; each kernel's rate is its share per launch over its own average
    launch time, against the matrix-core peak of its own type (the Gram
    products and X <- XV run on float32 or float64 MFMA)."""
    def share(kernels, steps):
        n = sum(kernels.get(nm, {}).get("launches", 0) for nm in JACOBI_KERNELS)
        return svd_flops * steps / n if n else None
    return {nm: ("mfma64" if nm.endswith("f64") else "mfma", share) for nm in JACOBI_KERNELS}


def per_launch(name, bytes_per_step):
    """units per launch of a kernel whose launches in a step differ in size:
    the step's algorithmic total over its launches"""
    def units(kernels, steps):
        n = kernels.get(name, {}).get("launches", 0) / max(1, steps)
        return bytes_per_step / n if n else None
    return units


def qprod_models(n1, m, n2, n3, p, backward):
    """HBM models of the transforms and dQ products of one qprod step (float32):
    every tensor a launch reads or writes, once."""
    hat = 4.0 * (n1 * m + m * n2) * (n3 + p) + 8.0 * n3 * p            # A and B to the transform domain
    unhat = 4.0 * n1 * n2 * (p + n3) + 4.0 * n3 * p                    # C back
    models = {"facewise_gemm": ("mfma", 2.0 * n1 * m * n2 * p)}
    if backward:
        # the backward transforms A and B again (their transforms are not
        # kept), and G
        hat = 2.0 * hat + 4.0 * n1 * n2 * (n3 + p) + 4.0 * n3 * p
        unhat += 4.0 * (n1 * m + m * n2) * (p + n3) + 8.0 * n3 * p      # dA, dB back
        dq = 4.0 * (p + n3) * (n1 * n2 + n1 * m + m * n2)               # the three dQ products' operands
        models["dq_gemm"] = ("hbm", per_launch("dq_gemm", dq))
    models["hat"] = ("hbm", per_launch("hat", hat))
    models["unhat"] = ("hbm", per_launch("unhat", unhat))
    return models


def host_of(X):
    """face-major device tensor -> numpy face-major storage (n3, n2, n1)"""
    return X.permute(2, 1, 0).contiguous().cpu().numpy()


def oracle_mod():
    import oracle
    return oracle


def tsvdq_cpu_case(Al, Qn, k):
    def run():
        o = oracle_mod()
        o.check_q(Qn)
        o.tsvdq(Al, Qn, k)
    return run, "check_q + tsvdq with A_k, spatial factors"


def workload_tsvdq(pq, torch, A_dev, Q_dev, k, a_bytes, name, prec):
    n1, n2, n3 = A_dev.shape
    p = Q_dev.shape[1]
    N = n1 * n2

    def step():
        pq.check_q(Q_dev)
        return pq.tsvdq(A_dev, Q_dev, k, prec=prec, spatial=True, approx=True)

    flops = (2.0 * N * n3 * p                         # transform
             + svd_nominal_flops(n1, n2, p)           # facewise SVD (nominal)
             + 2.0 * N * k * p * 2                    # factor + approximation products
             + 2.0 * N * n3 * p                       # A_k back to the spatial domain
             + 2.0 * (n1 + n2 + 1) * k * n3 * p)      # spatial factors
    models = {
        "hat": ("hbm", a_bytes * N * n3 + 4.0 * N * p + 4.0 * n3 * p),
        "unhat": ("hbm", None),   # several launches of different sizes
    }
    models.update(jacobi_models(svd_nominal_flops(n1, n2, p)))
    info = {"workload": name, "n1": n1, "n2": n2, "n3": n3, "p": p, "k": k}
    return step, flops, info, models


def host_info():
    """CPU model and BLAS build of this host, for the baseline's record."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        for d in threadpool_info():
            if d.get("user_api") == "blas":
                blas = f"{d.get('internal_api')} {d.get('version')} ({d.get('threading_layer', '')})"
                break
    except Exception:  # threadpoolctl missing
        pass
    return {"cpu_model": model, "blas": blas, "numpy": np.__version__, "nproc": os.cpu_count()}


def cpu_baseline(cpu_case, flops, seconds):
    """The float64 oracle timed on this host: a bounded sample of the same
    workload with every BLAS thread, then with one thread (half the budget
    each).  cpu_case is (run, description) for a callable that runs one full
    pass, or ("per-instance", factory, description) for one whose calls each
    time one instance and return (seconds, flops)."""
    from threadpoolctl import threadpool_limits

    def sample(budget):
        if cpu_case[0] == "per-instance":
            run = cpu_case[1]()
            t_cpu, fl, n = 0.0, 0.0, 0
            t_start = time.time()
            while time.time() - t_start < budget or n == 0:
                dt, f = run()
                t_cpu += dt
                fl += f
                n += 1
            return fl / t_cpu / 1e9, f"the first {n} instances (qprod + tSVDQ each), {t_cpu:.1f}s"
        run = cpu_case[0]
        run()  # warm-up
        reps, t_cpu = 0, 0.0
        t_start = time.time()
        while time.time() - t_start < budget or reps == 0:
            t1 = time.time()
            run()
            t_cpu += time.time() - t1
            reps += 1
        return flops * reps / t_cpu / 1e9, f"{reps} full passes of the same workload, {t_cpu:.1f}s"

    what = cpu_case[-1]
    cores = blas_threads()
    v_all, s_all = sample(0.5 * seconds)
    with threadpool_limits(limits=1, user_api="blas"):
        v_one, s_one = sample(0.5 * seconds)
    cpu = {"value": round(v_all, 4), "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
           "sample": f"{s_all} ({what}), float64 numpy/LAPACK on {cores} threads",
           "one_core": {"value": round(v_one, 4), "cores": 1, "sample": s_one}}
    cpu.update(host_info())
    log(f"cpu oracle: {cpu['value']} GFLOP/s on {cores} threads, {v_one:.4f} on one "
        f"({cpu['cpu_model']}, {cpu['blas']})")
    return cpu


def timed(torch, stream, fn, steps, warmup, lib):
    """ms per call of fn over `steps` calls after `warmup` calls (the
    autotuner on during the warm-up), between two events on the stream."""
    lib.pq_autotune_enable(1)
    for _ in range(max(1, warmup)):
        out = fn()
    torch.cuda.synchronize()
    lib.pq_autotune_enable(0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        out = fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, out


def rel_err(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))


def compare_forms(pq, torch, dev, up, args, insts, batch, shapes):
    """What the metric compares: the batched form against the plain float32
    path (sequential unbatched calls on the same instances), and the
    compensated split-bfloat16 forms against float32, each with its relative
    Frobenius error against the float64 oracle; plain bfloat16's error is
    reported as a number."""
    from paper_2409_19402_amd import _lib, synth
    import oracle
    lib = _lib.load()
    stream = torch.cuda.current_stream(dev)
    out = {}

    # the batched results against the oracle on four instances: the two
    # smallest and the two largest by element count
    sizes = [sh["n1"] * sh["n2"] * sh["n3"] for sh in shapes]
    order = [int(i) for i in np.argsort(sizes)]
    sample = order[:2] + order[-2:]
    e_c, e_s, e_a = 0.0, 0.0, 0.0
    for i in sample:
        sh, o = shapes[i], batch.outputs[i]
        c = synth.batched_instance(4, i, sh)
        Al, Bl = synth.logical(c["A"]), synth.logical(c["B"])
        ref = oracle.tsvdq(Al, c["Q"], sh["k"])
        U, s_, V = (o[x].double().cpu().numpy() for x in ("Uhat", "s", "Vhat"))
        e_c = max(e_c, rel_err(o["C"].double().cpu().numpy(), oracle.qprod(Al, Bl, c["Q"])))
        e_s = max(e_s, rel_err(s_, ref.s))
        e_a = max(e_a, rel_err(np.einsum("ijl,jl,mjl->iml", U, s_, V),
                               np.einsum("ijl,jl,mjl->iml", ref.Uhat, ref.s, ref.Vhat)))
    out["batched_rel_err_vs_oracle"] = {"instances": sample, "C": e_c, "s": e_s, "facewise_A_k": e_a}
    log(f"batched vs oracle on instances {sample}: C {e_c:.2e}, s {e_s:.2e}, facewise A_k {e_a:.2e}")

    # the hyperspectral-shaped tSVDQ: float32 transform vs split-bfloat16 x3
    # (and plain bfloat16, reported), whole step as the hyper workload times it
    c = synth.hyperspectral_case()
    A = pq.from_storage(torch.from_numpy(c["A_bits"].view(np.int16)).to(dev).view(torch.bfloat16))
    Q = torch.from_numpy(c["Q"]).to(dev)
    k = c["k"]
    ref = oracle.tsvdq(synth.logical(c["A"]), c["Q"], k)
    hyper = {}
    for prec in ("default", "bf16x3", "bf16"):
        ms, r = timed(torch, stream, lambda: (pq.check_q(Q), pq.tsvdq(A, Q, k, prec=prec, spatial=True,
                                                                        approx=True))[1],
                      5, 2, lib)
        err = rel_err(r.Ak.double().cpu().numpy(), ref.Ak)
        s_err = rel_err(r.s.double().cpu().numpy(), ref.s)
        name = "fp32" if prec == "default" else prec
        hyper[name] = {"ms_per_step": round(ms, 4), "rel_err_A_k": err, "rel_err_s": s_err}
        log(f"hyperspectral tSVDQ {name}: {ms:.3f} ms/step, A_k rel err {err:.2e}, s rel err {s_err:.2e}")
    ref_h = oracle.hat(synth.logical(c["A"]), c["Q"])
    for prec in ("default", "bf16x3", "bf16"):
        ms, Ah = timed(torch, stream, lambda: pq.hat(A, Q, prec=prec), 20, 3, lib)
        name = "fp32" if prec == "default" else prec
        hyper[name]["hat_us"] = round(1000 * ms, 2)
        hyper[name]["hat_rel_err"] = rel_err(Ah.double().cpu().numpy(), ref_h)
    hyper["bf16x3_speedup_vs_fp32"] = round(hyper["fp32"]["ms_per_step"] / hyper["bf16x3"]["ms_per_step"], 4)
    out["hyperspectral_tsvdq"] = hyper
    del A, c, ref, ref_h

    # the differentiation-shaped product A *_Q B (256x128x128 * 128x256x128,
    # p = 16) in the three precisions
    c = synth.differentiation_case()
    Ad, Bd = up(c["A"]), up(c["B"])
    Qd = torch.from_numpy(c["Q"]).to(dev)
    ref = oracle.qprod(synth.logical(c["A"]), synth.logical(c["B"]), c["Q"])
    qp = {}
    for prec in ("default", "bf16x3", "bf16"):
        ms, C = timed(torch, stream, lambda: pq.qprod(Ad, Bd, Qd, prec=prec), 50, 3, lib)
        name = "fp32" if prec == "default" else prec
        qp[name] = {"us_per_call": round(1000 * ms, 2), "rel_err": rel_err(C.double().cpu().numpy(), ref)}
        log(f"qprod {name}: {1000 * ms:.1f} us, rel err {qp[name]['rel_err']:.2e}")
    out["qprod_256x128x128"] = qp
    out["plain_bf16_rel_err"] = {"hyperspectral_hat": hyper["bf16"]["hat_rel_err"],
                                 "hyperspectral_A_k": hyper["bf16"]["rel_err_A_k"],
                                 "qprod_256x128x128": qp["bf16"]["rel_err"]}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU path, sharding over faces or rows, is not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2409_19402_amd import binding as pq
    from paper_2409_19402_amd import _lib, synth
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm device", file=sys.stderr)
        sys.exit(1)
    lib = _lib.load()
    dev = torch.device("cuda:0")

    def up(storage):
        return pq.from_storage(torch.from_numpy(np.ascontiguousarray(storage)).to(dev))

    def copy_rate(steps, warmup):
        """(ms per copy, GB/s) of a plain 512 MiB device copy (read + write)"""
        nbytes = 512 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(max(1, warmup)):
            dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        del src, dst
        return ms, 2 * nbytes / ms / 1e6

    if args.workload == "copy":
        # calibration of the HBM byte counters: a plain device copy of known size
        ms, gbs = copy_rate(args.steps, args.warmup)
        print(json.dumps({"workload": "copy", "bytes_read": 512 << 20, "bytes_written": 512 << 20,
                          "ms": ms, "GB/s": gbs}), flush=True)
        return

    t0 = time.time()
    cpu_case = None
    if args.workload == "video":
        c = synth.video_case()
        A, Q = up(c["A"]), torch.from_numpy(c["Q"]).to(dev)
        step, flops, info, models = workload_tsvdq(
            pq, torch, A, Q, c["k"], 4, "video-shaped tSVDQ 240x320x200 fp32, p=20, k=10", args.prec)
        dtype = "f32"
        cpu_case = tsvdq_cpu_case(synth.logical(c["A"]), c["Q"], c["k"])
    elif args.workload == "hyper":
        c = synth.hyperspectral_case()
        A = pq.from_storage(torch.from_numpy(c["A_bits"].view(np.int16)).to(dev).view(torch.bfloat16))
        Q = torch.from_numpy(c["Q"]).to(dev)
        step, flops, info, models = workload_tsvdq(
            pq, torch, A, Q, c["k"], 2, "hyperspectral-shaped tSVDQ 512x512x224 bf16, p=32, k=16",
            args.prec)
        dtype = "bf16-in/f32"
        cpu_case = tsvdq_cpu_case(synth.logical(c["A"]), c["Q"], c["k"])
    elif args.workload == "tiny":
        c = synth.tiny()
        A, Q = up(c["A"]), torch.from_numpy(c["Q"]).to(dev)
        step, flops, info, models = workload_tsvdq(
            pq, torch, A, Q, c["k"], 8, "tiny tSVDQ 32x24x16 fp64, p=4, k=5", "default")
        dtype = "f64"
        cpu_case = tsvdq_cpu_case(synth.logical(c["A"]), c["Q"], c["k"])
    elif args.workload == "svdii-video":
        c = synth.video_case()
        A, Q = up(c["A"]), torch.from_numpy(c["Q"]).to(dev)
        n1, n2, n3 = A.shape
        p, k = Q.shape[1], c["k"]
        N = n1 * n2
        kmax = min(n1, n2) // 4
        # gamma of Thm. 4.5: the transform-domain energy the rank-k tSVDQ keeps
        t_ = pq.tsvdq(A, Q, k)
        gamma = float((t_.s.double() ** 2).sum() / (pq.hat(A, Q).double() ** 2).sum())

        def step():
            pq.check_q(Q)
            return pq.svdii(A, Q, gamma, kmax=kmax, prec=args.prec, approx=True)
        flops = (2.0 * N * n3 * p + svd_nominal_flops(n1, n2, p)
                 + 2.0 * N * kmax * p * 2 + 2.0 * N * n3 * p)
        models = {"hat": ("hbm", 4.0 * N * n3 + 4.0 * N * p + 4.0 * n3 * p), "unhat": ("hbm", None)}
        models.update(jacobi_models(svd_nominal_flops(n1, n2, p)))
        info = {"workload": f"video-shaped *_Q-SVDII 240x320x200 fp32, p=20, gamma of rank-{k} tSVDQ, "
                            f"kmax={kmax}", "n1": n1, "n2": n2, "n3": n3, "p": p, "gamma": gamma,
                "kmax": kmax}
        dtype = "f32"
        Al, Qn = synth.logical(c["A"]), c["Q"]
        cpu_case = (lambda: (oracle_mod().check_q(Qn), oracle_mod().tsvdq_ii(Al, Qn, gamma)),
                    "check_q + tsvdq_ii with A_k")
    elif args.workload == "tsvdq-backward-video":
        c = synth.video_case()
        A, Q = up(c["A"]), torch.from_numpy(c["Q"]).to(dev)
        n1, n2, n3 = A.shape
        p, k = Q.shape[1], c["k"]
        N, L, S = n1 * n2, max(n1, n2), min(n1, n2)
        rng = np.random.default_rng(6)
        Gbar = up(rng.standard_normal((n3, n2, n1), dtype=np.float32))
        sbar = torch.from_numpy(rng.standard_normal((k, p)).astype(np.float32)).to(dev)

        def step():
            return pq.tsvdq_backward(A, Q, k, Gbar=Gbar, sbar=sbar)
        flops = (2.0 * N * n3 * p * 2                   # transforms of A and Gbar
                 + svd_nominal_flops(n1, n2, p)         # the recomputed facewise SVD
                 + 2.0 * L * S * S * p                  # M_t^T U
                 + 2.0 * p * (4 * L * S * k + 2 * S * S * k)  # the k-column products
                 + 2.0 * N * 2 * k * p                  # the face gradient
                 + 2.0 * N * k * p                      # transform-domain A_k
                 + 2.0 * N * n3 * p                     # dA back to the spatial domain
                 + 2.0 * 2 * N * n3 * p)                # the two dQ products
        models = {"hat": ("hbm", None), "unhat": ("hbm", None)}
        models.update(jacobi_models(svd_nominal_flops(n1, n2, p)))
        info = {"workload": "tSVDQ adjoint (dA, dQ of <Gbar, A_k> + <sbar, s>), video-shaped "
                            "240x320x200 fp32, p=20, k=10", "n1": n1, "n2": n2, "n3": n3, "p": p, "k": k}
        dtype = "f32"
        Al, Qn, Gl, sb = synth.logical(c["A"]), c["Q"], synth.logical(host_of(Gbar)), sbar.cpu().numpy()
        cpu_case = (lambda: oracle_mod().tsvdq_backward(Al, Qn, k, Gl, sb), "tsvdq_backward (float64 SVD perturbation)")
    elif args.workload in ("u3-video", "u3-video-f64"):
        c = synth.video_case()
        f64 = args.workload == "u3-video-f64"
        A_st = c["A"].astype(np.float64) if f64 else c["A"]
        A = up(A_st)
        n1, n2, n3 = A.shape
        p = 20
        N = n1 * n2

        def step():
            return pq.u3(A, p)
        flops = 2.0 * N * n3 * n3 + svd_nominal_flops(n3, n3, 1)
        models = {"u3_gram": ("mfma64" if f64 else "mfma", 2.0 * N * n3 * n3)}
        models.update(jacobi_models(svd_nominal_flops(n3, n3, 1)))
        info = {"workload": "Q = U3(:, 1:20) of the video-shaped 240x320x200 "
                            + ("cube in float64" if f64 else "fp32 cube"),
                "n1": n1, "n2": n2, "n3": n3, "p": p}
        dtype = "f64" if f64 else "f32"
        Al = synth.logical(A_st)
        cpu_case = (lambda: oracle_mod().u3(Al, p), "u3 (Gram eigen route of the oracle)")
    elif args.workload in ("hat-video", "hat-hyper", "proj-video"):
        if args.workload == "hat-hyper":
            c = synth.hyperspectral_case()
            A = pq.from_storage(torch.from_numpy(c["A_bits"].view(np.int16)).to(dev)
                                .view(torch.bfloat16))
            a_bytes, dtype, nm = 2, "bf16-in/f32", "transform A x_3 Q^T, 512x512x224 bf16 -> p=32"
        else:
            c = synth.video_case()
            A = up(c["A"])
            a_bytes, dtype, nm = 4, "f32", "transform A x_3 Q^T, 240x320x200 fp32 -> p=20"
        Q = torch.from_numpy(c["Q"]).to(dev)
        n1, n2, n3 = A.shape
        p = Q.shape[1]
        N = n1 * n2
        if args.workload == "proj-video":
            nm = "projection A x_3 Q Q^T, 240x320x200 fp32, p=20"

            def step():
                return pq.proj(A, Q, prec=args.prec)
            flops = 4.0 * N * n3 * p
            models = {"proj_fused": ("hbm", 2 * a_bytes * N * n3 + 4.0 * n3 * p)}
        else:
            def step():
                return pq.hat(A, Q, prec=args.prec)
            flops = 2.0 * N * n3 * p
            models = {"hat": ("hbm", a_bytes * N * n3 + 4.0 * N * p + 4.0 * n3 * p)}
        info = {"workload": nm, "n1": n1, "n2": n2, "n3": n3, "p": p}
    elif args.workload == "qprod":
        c = synth.differentiation_case()
        A, B = up(c["A"]), up(c["B"])
        Q = torch.from_numpy(c["Q"]).to(dev)
        n1, m, n3 = A.shape
        n2 = B.shape[1]
        p = Q.shape[1]

        def step():
            return pq.qprod(A, B, Q, prec=args.prec)
        flops = 2.0 * p * (n1 * m * n3 + m * n2 * n3 + n1 * m * n2 + n1 * n2 * n3)
        models = qprod_models(n1, m, n2, n3, p, backward=False)
        info = {"workload": "qprod 256x128x128 * 128x256x128 fp32, p=16", "n1": n1, "m": m,
                "n2": n2, "n3": n3, "p": p}
        dtype = "f32"
    elif args.workload == "facewise":
        # the facewise product (Def. 2.3) alone on the largest faces of the
        # batched workload: 32 faces of 512 x 512 times 512 x 512
        n1 = m = n2 = 512
        p = 32
        rng = np.random.default_rng(8)
        Ah, Bh = up(synth.gaussian(rng, n1, m, p)), up(synth.gaussian(rng, m, n2, p))

        def step():
            return pq.facewise(Ah, Bh, prec=args.prec)
        flops = 2.0 * n1 * m * n2 * p
        passes = {"default": 0, "fp32": 0, "bf16": 1, "bf16x3": 3, "bf16x6": 6}[args.prec]
        # float32 MFMA: the algorithmic flops against the float32 peak; the
        # split-bfloat16 modes: the bfloat16 products they execute (passes x
        # the algorithmic flops) against the bfloat16 peak
        models = {"facewise_gemm": ("mfma", flops) if passes == 0 else ("mfma_bf16", passes * flops)}
        info = {"workload": f"facewise product, {p} faces of {n1}x{m} times {m}x{n2}, fp32 data",
                "n1": n1, "m": m, "n2": n2, "p": p}
        dtype = "f32" if passes == 0 else "bf16"
    elif args.workload == "batched":
        shapes = synth.batched_shapes(count=args.count)
        insts, flops, cpu_insts = [], 0.0, []
        for i, sh in enumerate(shapes):
            c = synth.batched_instance(4, i, sh)
            insts.append(dict(A=up(c["A"]), B=up(c["B"]), Q=torch.from_numpy(c["Q"]).to(dev), k=sh["k"]))
            n1, n2, n3, n4, p, k = (sh[x] for x in ("n1", "n2", "n3", "n4", "p", "k"))
            f = (2.0 * p * (n1 * n2 * n3 + n2 * n4 * n3 + n1 * n2 * n4 + n1 * n4 * n3)   # qprod
                 + 2.0 * n1 * n2 * n3 * p + svd_nominal_flops(n1, n2, p))               # tSVDQ steps 2-3
            flops += f
            cpu_insts.append((i, sh, f))
        batch_box = {}

        def step():
            batch_box["b"].run()
            return batch_box["b"]

        def plan():
            if "b" in batch_box:
                batch_box["b"].close()
            batch_box["b"] = pq.batched(insts)
            return batch_box["b"]

        def unbatched():
            for x in insts:
                pq.qprod(x["A"], x["B"], x["Q"])
                pq.tsvdq(x["A"], x["Q"], x["k"])

        models = jacobi_models(sum(svd_nominal_flops(sh["n1"], sh["n2"], sh["p"]) for sh in shapes))
        info = {"workload": f"batched: {len(shapes)} uneven instances (qprod + rank-p/2 tSVDQ each), "
                            "n1,n2,n4 in [64,512], n3 in [32,256], p in [4,32], fp32",
                "instances": len(shapes),
                "a_elements": int(sum(sh["n1"] * sh["n2"] * sh["n3"] for sh in shapes)),
                "faces": int(sum(sh["p"] for sh in shapes))}
        dtype = "f32"

        def cpu_batched():
            import oracle
            state = {"i": 0}

            def run():
                # one instance per call, in order: check_q + qprod + tSVDQ
                j, sh, f = cpu_insts[state["i"] % len(cpu_insts)]
                state["i"] += 1
                c = synth.batched_instance(4, j, sh)
                Al, Bl = synth.logical(c["A"]), synth.logical(c["B"])
                t1 = time.time()
                oracle.check_q(c["Q"])
                oracle.qprod(Al, Bl, c["Q"])
                oracle.tsvdq(Al, c["Q"], sh["k"])
                return time.time() - t1, f
            return run
        cpu_case = ("per-instance", cpu_batched, "check_q + qprod + tSVDQ of the batch's instances in order")
    else:  # diff
        c = synth.differentiation_case()
        A = up(c["A"]).requires_grad_(True)
        B = up(c["B"]).requires_grad_(True)
        Q = torch.from_numpy(c["Q"]).to(dev).requires_grad_(True)
        T = up(c["T"])
        n1, m, n3 = A.shape
        n2 = B.shape[1]
        p = Q.shape[1]
        G = pq.empty(n1, n2, n3, device=dev)

        def step():
            C = pq.QProd.apply(A, B, Q, args.prec)
            with torch.no_grad():  # the loss gradient G = 2 (C - T)
                G.copy_(C)
                G.sub_(T).mul_(2.0)
            return pq.qprod_backward(G, A.detach(), B.detach(), Q.detach())

        fw = 2.0 * p * (n1 * m * n3 + m * n2 * n3 + n1 * m * n2 + n1 * n2 * n3)
        bw = (2.0 * n1 * n2 * n3 * p + 4.0 * n1 * m * n2 * p + 2.0 * n3 * p * (n1 * m + m * n2)
              + 2.0 * n3 * p * (n1 * n2 + n1 * m + m * n2) + 2.0 * p * (n1 * m * n3 + m * n2 * n3)
              + 2.0 * p * n1 * m * n2)
        flops = fw + bw
        models = qprod_models(n1, m, n2, n3, p, backward=True)
        info = {"workload": "qprod forward+backward 256x128x128 * 128x256x128 fp32, p=16",
                "n1": n1, "m": m, "n2": n2, "n3": n3, "p": p}
        dtype = "f32"
    log(f"inputs ready in {time.time() - t0:.1f}s: {info['workload']}")

    stream = torch.cuda.current_stream(dev)
    # warm-up; the first pass also lets the library's autotuner time the
    # candidate launch configurations of every kernel shape in the step
    lib.pq_autotune_enable(1)
    if args.workload == "batched":
        unbatched()  # tunes the per-instance launch shapes of the plain path
        plan()       # eager pass + graph capture
    for _ in range(max(1, args.warmup)):
        out = step()
    torch.cuda.synchronize()
    lib.pq_autotune_enable(0)
    log(f"warmup done ({lib.pq_autotune_entries()} tuned launch shapes)")
    # cycles of torch's bounded spin kernel per millisecond on this device
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    torch.cuda._sleep(2_000_000)
    e1.record(stream)
    torch.cuda.synchronize()
    spin_cycles_per_ms = 2_000_000 / max(1e-3, e0.elapsed_time(e1))
    # the host time to enqueue one step (tuned, nothing to wait for)
    t_host = time.perf_counter()
    out = step()
    t_host = time.perf_counter() - t_host
    torch.cuda.synchronize()

    # the timed region: K steps between two events on the launch stream, with
    # an event after each step for the spread of single-step times
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    ev0.record(stream)
    for i in range(args.steps):
        out = step()
        marks[i].record(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    singles = [ev0.elapsed_time(marks[0])] + [marks[i - 1].elapsed_time(marks[i]) for i in range(1, args.steps)]
    q10, q50, q90 = (float(np.percentile(singles, q)) for q in (10, 50, 90))
    log(f"timed {args.steps} steps: {ms_per_step:.4f} ms/step (single steps p10 {q10:.4f}, median {q50:.4f}, "
        f"p90 {q90:.4f} ms)")

    extra_batched = {}
    if args.workload == "batched":
        # the same work as sequential unbatched calls (the plain fp32 path),
        # three passes after the warm-up's tuned one
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(3):
            unbatched()
        ev1.record(stream)
        torch.cuda.synchronize()
        ub = ev0.elapsed_time(ev1) / 3
        extra_batched = {"fp32_unbatched_ms_per_step": round(ub, 4),
                         "batched_speedup_vs_fp32_unbatched": round(ub / ms_per_step, 3),
                         "workspace_GB": round(out.workspace_bytes / 1e9, 3)}
        log(f"unbatched: {ub:.3f} ms/step, batched graph {ms_per_step:.3f} ms/step")

    # a second pass of the same K steps with the library's per-launch
    # profiler on (HIP events around every launch, on the launch stream);
    # a captured graph records no events, so the batched workload profiles
    # the eager pass of a fresh plan instead
    lib.pq_profile_reset()
    lib.pq_profile_enable(1)
    if args.workload == "batched":
        out = plan()
        prof_steps = 1
    else:
        # A step whose kernels finish before the host has enqueued the next
        # launch leaves the GPU idle between a launch's start event and the
        # kernel itself, and the event pair would time the host.  A bounded
        # spin kernel queued first holds the stream for longer than the host
        # needs to enqueue the K steps, so every event pair brackets its
        # kernel alone (the timed region above keeps the host in the loop).
        spin_ms = min(200.0, 4.0 * args.steps * t_host * 1e3 + 2.0)
        torch.cuda._sleep(int(spin_ms * spin_cycles_per_ms))
        for _ in range(args.steps):
            out = step()
        prof_steps = args.steps
    torch.cuda.synchronize()
    lib.pq_profile_enable(0)

    # per-kernel durations from the library's own events on the launch stream
    import ctypes
    buf = ctypes.create_string_buffer(4096)
    lib.pq_profile_names(buf, 4096)
    kernels = {}
    for nm in [x for x in buf.value.decode().split(",") if x]:
        t = ctypes.c_double()
        n = ctypes.c_int()
        lib.pq_profile_query(nm.encode(), ctypes.byref(t), ctypes.byref(n))
        kernels[nm] = {"total_ms": t.value, "launches": n.value,
                       "avg_us": 1000.0 * t.value / max(1, n.value)}
    lib.pq_profile_reset()
    for nm, d in sorted(kernels.items(), key=lambda kv: -kv[1]["total_ms"]):
        log(f"  {nm:18s} {d['total_ms'] / prof_steps * 1000:10.1f} us/step  "
            f"{d['launches'] // max(1, prof_steps)} launches/step  avg {d['avg_us']:.1f} us")

    # dominant kernel and its roofline
    dom = max(kernels.items(), key=lambda kv: kv[1]["total_ms"])[0] if kernels else None
    roof = None
    if dom is not None:
        bound, units = models.get(dom, ("hbm", None))
        if callable(units):
            units = units(kernels, prof_steps)
        avg_s = kernels[dom]["avg_us"] * 1e-6
        if units is not None and avg_s > 0:
            if bound == "hbm":
                achieved, peak, unit = units / avg_s / 1e9, HBM_PEAK_GBS, "GB/s"
            elif bound == "mfma64":
                achieved, peak, unit = units / avg_s / 1e12, FP64_MFMA_PEAK, "TFLOP/s"
            elif bound == "mfma_bf16":
                achieved, peak, unit = units / avg_s / 1e12, BF16_MFMA_PEAK, "TFLOP/s"
            else:
                achieved, peak, unit = units / avg_s / 1e12, FP32_MFMA_PEAK, "TFLOP/s"
            roof = {"kernel": dom, "bound": "mfma" if bound in ("mfma64", "mfma_bf16") else bound,
                    "achieved": round(achieved, 4), "peak": peak,
                    "unit": unit, "frac": round(achieved / peak, 6),
                    "traffic": TRAFFIC_BYTES.get((args.workload, args.prec, dom)),
                    "avg_us": round(kernels[dom]["avg_us"], 3)}
            if bound == "hbm":
                # the same rate against what a plain device copy reaches here
                _, copy_gbs = copy_rate(5, 2)
                roof["measured_peak"] = round(copy_gbs, 1)
                roof["frac_measured"] = round(achieved / copy_gbs, 6)

    extra = {}
    if args.workload == "svdii-video":
        rho = out.rho.cpu()
        Af = A.float()
        re = (torch.linalg.vector_norm((Af - out.Ak).reshape(-1)) /
              torch.linalg.vector_norm(Af.reshape(-1))).item()
        extra = {"relative_error_A_k": re, "implicit_rank": int(rho.sum()), "rho_max": int(rho.max()),
                 "rho_min": int(rho.min()), "tsvdq_implicit_rank": k * p}
        log(f"RE(A_k) = {re:.6e}, rho {rho.tolist()}")
    if args.workload in ("video", "hyper", "tiny"):
        Ak = out.Ak
        Af = A.float() if A.dtype != torch.float64 else A
        re = (torch.linalg.vector_norm((Af - Ak).reshape(-1)) /
              torch.linalg.vector_norm(Af.reshape(-1))).item()
        inf = out.info.cpu().tolist()
        extra = {"relative_error_A_k": re, "jacobi_sweeps_max": inf[0],
                 "unconverged_faces": inf[1], "jacobi_sweeps_total": inf[2]}
        log(f"RE(A_k) = {re:.6e}, sweeps max {inf[0]}, total {inf[2]}, unconverged {inf[1]}")

    value = flops / (ms_per_step * 1e-3) / 1e9

    # CPU oracle baseline (float64, this host's cores), a bounded sample
    cpu = None
    if not args.no_cpu_baseline and cpu_case is not None:
        cpu = cpu_baseline(cpu_case, flops, args.cpu_seconds)

    if args.workload == "batched" and not args.no_compare:
        extra_batched.update(compare_forms(pq, torch, dev, up, args, insts, out, shapes))

    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "ms_per_step_quantiles": {"p10": round(q10, 5), "p50": round(q50, 5), "p90": round(q90, 5)},
        "host_enqueue_ms_per_step": round(t_host * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": dict(info, prec=args.prec, **extra, **extra_batched),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    detail = {"kernels_per_step_us": {k2: v["total_ms"] / prof_steps * 1000 for k2, v in kernels.items()},
              "kernels": kernels, "flops_per_step": flops, "line": line}
    if args.details:
        with open(args.details, "w") as fh:
            json.dump(detail, fh, indent=1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
