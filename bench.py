"""Benchmark: HODLR-QDWH spectral projectors per second on one MI355X.

One step = one call of spectral_projector (Algorithm hQDWH: scalar setup, structured first
iteration, Cholesky iterations, symmetrisation) on a band already resident in HBM.  Prints one JSON
line.  Default workload: symmetric banded n = 16384, b = 8, N(0,1) band entries mirrored plus
4i/n on the diagonal, mu between lambda_{n/2} and lambda_{n/2+1}, leaf 128, tol 1e-10, FP64.

`value` is the FP64 projectors per second of that workload.  The line also carries the legs of the
comparison the metric asks for, measured in the same run: the same matrix in mixed precision (FP32
middle iterations) with its error against the FP64 projector, the FP64 solve without the rank
predictor, and a batch of independent matrices of the batched workload's generator (n_i ~
U{2048..16384}, b_i ~ U{1..16}) in FP64 and in mixed precision; Zolo-pd (the two-step alternative
that Sec. 2.1 cites) on the same matrix with its difference to the QDWH projector; plus the
matrix-core utilisation (flops issued as MFMA instructions / time / peak of their precision) of the
timed steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (maker, b, leaf, tol)
    "banded-n16384-b8": (lambda: __import__("workloads").banded_normal(16384, 8, 0), 8, 128, 1e-10),
    "tridiag-n1024": (lambda: __import__("workloads").tridiag_uniform(1024, 0), 1, 64, 1e-10),
    "banded-n4096-b8": (lambda: __import__("workloads").banded_normal(4096, 8, 0), 8, 128, 1e-10),
    "metallic-n32768": (lambda: __import__("workloads").tridiag_metallic(32768, 0), 1, 256, 1e-10),
    "tridiag-n100000": (lambda: __import__("workloads").tridiag_uniform(100000, 0), 1, 256, 1e-8),
}
# batched: count independent banded matrices, n_i ~ U{2048..16384}, b_i ~ U{1..16}, leaf 128, tol 1e-10
BATCHED = {"batched-256": 256, "batched-64": 64, "batched-16": 16}
DEFAULT = "banded-n16384-b8"
LEG_BATCH = 16  # members of the batched legs of the default line
METRIC = "HODLR-QDWH Π/s at ‖Π−Π_oracle‖₂≤1e-8: mixed+batched vs FP64; MFMA util %"

# MI355X peaks: FP64 MFMA 78.6 TFLOP/s, FP32 MFMA 157.3 TFLOP/s (dense); FP64 vector ALU
# 256 CUs x 2.4 GHz x 128 flop/clk = 78.6 TFLOP/s
PEAK_FP64_MFMA = 78.6
PEAK_FP32_MFMA = 157.3
PEAK_FP64_ALU = 78.6
KERNEL_NAMES = {"gemm": "k_gemm", "tsqr": "k_qr_stage", "core_svd": "k_svd", "leaf_cholesky": "k_chol_inv",
                "leaf_inverse": "k_trtri", "stack": "k_stack", "leaf_elementwise": "k_leaf_axpy", "other": "misc"}


def band_matvec_torch(band, X):
    """Y = A X for the symmetric band matrix held in lower band storage (device tensors)."""
    n, ld = band.shape
    Y = band[:, 0:1] * X
    for i in range(1, ld):
        c = band[: n - i, i: i + 1]
        Y[i:] += c * X[: n - i]
        Y[: n - i] += c * X[i:]
    return Y


def properties(P, band, mu, seed=0):
    """At-any-size checks of a projector: idempotency, commutation with A, sign of the spectrum."""
    import torch
    n = band.shape[0]
    g = torch.Generator(device="cuda").manual_seed(seed)
    X = torch.randn((n, 4), generator=g, dtype=torch.float64, device="cuda")
    PX = P.apply(X)
    PPX = P.apply(PX.contiguous())
    AX = band_matvec_torch(band, X)
    APX = band_matvec_torch(band, PX)
    PAX = P.apply(AX.contiguous())
    idem = float((PPX - PX).norm() / X.norm())
    comm = float((APX - PAX).norm() / X.norm())
    # Rayleigh quotients of A - mu on range(P) must be negative, on range(I-P) positive
    neg = float(((PX * (APX - mu * PX)).sum(0) / (PX * PX).sum(0)).max())
    QX = X - PX
    AQX = AX - APX
    pos = float(((QX * (AQX - mu * QX)).sum(0) / (QX * QX).sum(0)).min())
    return {"idempotency": idem, "commutation": comm, "rayleigh_below_mu": neg, "rayleigh_above_mu": pos}


def difference_norm(P1, P2, n, steps=40, seed=1):
    """||P1 - P2||_2 by symmetric Lanczos with full reorthogonalisation on the device (both applied
    through the library)."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    q = torch.randn((n, 1), generator=g, dtype=torch.float64, device="cuda")
    q /= q.norm()
    Q = [q]
    al, be = [], []
    beta, qp = 0.0, torch.zeros_like(q)
    for _ in range(steps):
        wv = P1.apply(q) - P2.apply(q)
        a = float((q * wv).sum())
        wv = wv - a * q - beta * qp
        Qm = torch.cat(Q, 1)
        wv -= Qm @ (Qm.T @ wv)
        wv -= Qm @ (Qm.T @ wv)
        al.append(a)
        beta = float(wv.norm())
        if beta < 1e-300:
            break
        be.append(beta)
        qp, q = q, wv / beta
        Q.append(q)
    k = len(al)
    T = np.diag(al) + np.diag(be[: k - 1], 1) + np.diag(be[: k - 1], -1)
    return float(np.max(np.abs(np.linalg.eigvalsh(T))))


def measured_traffic(workload, kernel):
    """HBM bytes per dispatch of `kernel` from the committed counter summary of `workload`, or None when
    there is none or the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic-{kernel}-{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split(None, 1)
            kv[k] = v
    src = os.path.join(ROOT, "paper_1608_01164_amd", "csrc", "kernels.hip")
    if kv.get("kernel") != kernel or hashlib.sha256(open(src, "rb").read()).hexdigest() != kv.get("source_sha256"):
        return None
    kib = float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"]) + \
        float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"])
    return kib * 1024.0


def kernel_table(prof):
    kern = {}
    for k, v in prof.items():
        if v["launches"]:
            kern[k] = {"kernel": KERNEL_NAMES[k], "launches": v["launches"], "ms_total": v["ms"],
                       "ms_avg": v["ms"] / v["launches"], "gflop_per_launch": v["flops"] / v["launches"] / 1e9,
                       "tflops": v["flops"] / max(v["ms"], 1e-9) / 1e9}
    return kern


def roofline(prof, workload=None):
    """Roofline entry of the kernel class with the largest measured time (HIP events on the streams the
    library launches it on, over the timed steps)."""
    kern = kernel_table(prof)
    dom = max(kern, key=lambda k: kern[k]["ms_total"])
    d = kern[dom]
    bound = "mfma" if dom == "gemm" else "alu"
    peak = PEAK_FP64_MFMA if bound == "mfma" else PEAK_FP64_ALU
    achieved = d["tflops"]
    return {"kernel": d["kernel"], "bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": measured_traffic(workload, d["kernel"]) if workload else None,
            "traffic_unit": "bytes per launch", "avg_launch_ms": d["ms_avg"],
            "flops_per_launch": d["gflop_per_launch"] * 1e9}


def mfma_util(mf, seconds):
    """Matrix-core utilisation: flops issued as MFMA instructions over the elapsed time, against the
    dense peak of their precision."""
    t64 = mf["fp64"] / seconds / 1e12
    t32 = mf["fp32"] / seconds / 1e12
    return {"fp64_tflops": t64, "fp64_util_pct": 100.0 * t64 / PEAK_FP64_MFMA,
            "fp32_tflops": t32, "fp32_util_pct": 100.0 * t32 / PEAK_FP32_MFMA}


def timed_classes(prof_w):
    """Kernel classes whose launches get HIP events in the timed steps: the class with the largest time
    in the fully timed warmup step (events on every launch of a long chain of short kernels cost host
    time of their own), or every class when there was no warmup."""
    if prof_w is None:
        return None
    busy = {k: v["ms"] for k, v in prof_w.items() if v["launches"]}
    return [max(busy, key=busy.get)] if busy else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ab, b, nu, budget_s=20.0):
    """The oracle on a bounded sample: m eigenpairs (bisection + inverse iteration) and their share of
    Pi = V V^T, extrapolated linearly to all nu eigenpairs."""
    from oracle import eig
    n = ab.shape[0]
    t0 = time.perf_counter()
    m = 8
    spent = 0.0
    while True:
        t = time.perf_counter()
        lam = eig.eigenvalues(ab, 1, m)
        V = eig.eigenvectors(ab, lam)
        V @ V.T
        spent = time.perf_counter() - t
        if spent > budget_s / 4 or m >= nu:
            break
        m *= 2
    per_pair = spent / m
    total = per_pair * nu
    return {"value": 1.0 / total, "unit": "Π/s", "cores": eig.num_threads(), "cpu": cpu_model(), "kind": "oracle",
            "sample": f"{m} of {nu} eigenpairs (inertia bisection + inverse iteration + V V^T share) in "
                      f"{spent:.2f} s, extrapolated linearly to nu={nu}; n={n}, b={b}",
            "sample_seconds": spent, "extrapolated_seconds": total, "wall_s": time.perf_counter() - t0}


def _predictor(no_predictor):
    if no_predictor:
        return None
    from paper_1608_01164_amd import predictor as hp
    return hp.load() if os.path.exists(hp.DEFAULT_PATH) else None


def timed_single(hq, band, b, mu, leaf, tol, pred, precision, steps, warmup, tag, method="qdwh"):
    """Warmup then `steps` timed calls (no timers); returns (Π/s, last projector, last info)."""
    import torch
    for i in range(warmup):
        P, info = hq.spectral_projector(band, b, mu, leaf=leaf, tol=tol, predictor=pred, precision=precision,
                                        method=method)
        P.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = None
    for i in range(steps):
        if P is not None:
            P.close()
        P, info = hq.spectral_projector(band, b, mu, leaf=leaf, tol=tol, predictor=pred, precision=precision,
                                        method=method)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"# leg {tag}: {steps} steps, {dt / steps:.3f} s per projector, K={info['iters']}, "
          f"fp32 iterations {info['fp32_iter']}, redo {info['redo_count']}", file=sys.stderr, flush=True)
    return steps / dt, P, info


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS) + sorted(BATCHED))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="only the main workload (no mixed / batched legs)")
    ap.add_argument("--no-profile", action="store_true", help="disable the library's per-launch kernel timers")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="mixed: middle QDWH iterations in FP32 (GEMM on FP32 MFMA, FP32 TSQR and core SVD)")
    ap.add_argument("--method", default="qdwh", choices=["qdwh", "zolo"],
                    help="zolo: Zolo-pd (two Zolotarev steps, FP64) instead of the QDWH iterations")
    ap.add_argument("--no-predictor", action="store_true",
                    help="capacities from the previous iterate's ranks instead of the trained rank predictor")
    ap.add_argument("--graph", action="store_true",
                    help="launch each Cholesky iteration as one captured HIP graph")
    ap.add_argument("--iter-log", metavar="PATH",
                    help="append one JSON line per iteration of every timed step to PATH (weights, rank, seconds)")
    ap.add_argument("--sweep", choices=["nmin", "memory", "scaling", "breakeven", "hmatrix", "solve"],
                    help="one of the paper's timing/memory experiments on Sec. 6.1 test matrices instead of "
                         "the benchmark line (JSON lines, one per case)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); sharding "
              "matrices or subtrees across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1608_01164_amd as hq

    if args.sweep:
        return SWEEPS[args.sweep](hq)
    if args.workload in BATCHED:
        return main_batched(args, BATCHED[args.workload])
    maker, b, leaf, tol = WORKLOADS[args.workload]
    pred = _predictor(args.no_predictor)
    ab = maker()
    n = ab.shape[0]
    nu = n // 2
    mu, gap = hq.shift_for_count(ab, b, nu)
    band = torch.from_numpy(np.ascontiguousarray(ab)).cuda()
    torch.cuda.synchronize()
    print(f"# workload {args.workload}: n={n} b={b} leaf={leaf} tol={tol} mu={mu:.6e} gap={gap:.3e}",
          file=sys.stderr, flush=True)
    info = None
    prof_w = None
    for i in range(args.warmup):
        last = i == args.warmup - 1 and not args.no_profile
        if last:
            hq.profile(True)
        P, info = hq.spectral_projector(band, b, mu, leaf=leaf, tol=tol, predictor=pred, precision=args.precision,
                                        graph=args.graph, method=args.method)
        P.close()
        if last:
            prof_w = hq.profile_read()
            hq.profile(False)
        print(f"# warmup {i}: {info['seconds']:.3f} s, K={info['iters']}, max rank {info['max_rank']}",
              file=sys.stderr, flush=True)
    if not args.no_profile:
        hq.profile(True, classes=timed_classes(prof_w))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    P = None
    for i in range(args.steps):
        if P is not None:
            P.close()
        P, info = hq.spectral_projector(band, b, mu, leaf=leaf, tol=tol, predictor=pred, precision=args.precision,
                                        graph=args.graph, method=args.method)
        infos.append(info)
        print(f"# step {i}: {info['seconds']:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if args.iter_log:  # written after the timed region
        with open(args.iter_log, "a") as f:
            for i, inf in enumerate(infos):
                for rec in hq.iteration_records(inf, workload=args.workload, step=i, method=args.method,
                                                precision=args.precision):
                    f.write(json.dumps(rec) + "\n")
    svd_stats = hq.binding.profile_svd() if not args.no_profile else None
    prof = hq.profile_read() if not args.no_profile else None
    mf = hq.binding.profile_mfma() if not args.no_profile else None
    if not args.no_profile:
        hq.profile(False)
    ms = 1e3 * (t1 - t0) / args.steps
    value = args.steps / (t1 - t0)
    props = properties(P, band, mu)
    out = {
        "metric": METRIC, "value": value, "unit": "Π/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f64+f32", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "b": b, "leaf": leaf, "tol": tol, "nu": nu, "mu": mu,
                   "gap": gap, "precision": args.precision, "method": args.method, "parallelism": "single-gpu",
                   "capacities": "predictor" if pred is not None else "previous ranks"},
        "iters": info["iters"], "max_rank": info["max_rank"], "launches": info["launches"],
        "setup_s": info["setup_seconds"], "givens_s": info["givens_seconds"], "peak_bytes": info["peak_bytes"],
        "redo_count": info["redo_count"],
        "checks": props,
    }
    if prof is not None:
        out["roofline"] = roofline(prof, args.workload)
        out["roofline"]["measured_over"] = "timed steps (HIP events on the dominant class's launches only)"
        out["mfma"] = mfma_util(mf, t1 - t0)
        out["kernels"] = kernel_table(prof_w if prof_w is not None else prof)
        out["kernels_source"] = "last warmup step, every kernel class timed" if prof_w is not None else "timed steps"
        out["core_svd_phases"] = svd_stats
    if not args.no_legs and args.workload == DEFAULT and args.precision == "fp64" and args.method == "qdwh":
        out["legs"] = legs(hq, band, b, mu, leaf, tol, pred, P, value, n)
    P.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ab, b, nu)
    print(json.dumps(out), flush=True)


def legs(hq, band, b, mu, leaf, tol, pred, P64, value64, n):
    """The comparison legs of the metric on the same GPU (short runs, no timers)."""
    out = {}
    # the same matrix with FP32 middle iterations; its error against the FP64 projector (which the
    # parity tests hold to 1e-8 against the oracle)
    v, Pm, im = timed_single(hq, band, b, mu, leaf, tol, pred, "mixed", 3, 1, "mixed")
    out["mixed"] = {"value": v, "unit": "Π/s", "vs_fp64": v / value64, "iters": im["iters"],
                    "fp32_iterations": im["fp32_iter"], "redo_count": im["redo_count"],
                    "err_vs_fp64_2norm": difference_norm(Pm, P64, n)}
    Pm.close()
    v, Pn, inn = timed_single(hq, band, b, mu, leaf, tol, None, "fp64", 3, 1, "fp64-no-predictor")
    out["fp64_no_predictor"] = {"value": v, "unit": "Π/s", "predictor_speedup": value64 / v,
                                "redo_count": inn["redo_count"], "capacity_columns": inn["capacity_columns"]}
    Pn.close()
    out["batched"] = batched_legs(hq, LEG_BATCH, pred)
    # Zolo-pd on the same matrix (two steps of degree r instead of the QDWH iterations)
    v, Pz, iz = timed_single(hq, band, b, mu, leaf, tol, None, "fp64", 2, 1, "zolo", method="zolo")
    out["zolo"] = {"value": v, "unit": "Π/s", "vs_qdwh": v / value64, "steps": iz["iters"], "r": iz["zolo_r"],
                   "redo_count": iz["redo_count"], "max_rank": iz["max_rank"], "peak_bytes": iz["peak_bytes"],
                   "err_vs_qdwh_2norm": difference_norm(Pz, P64, n)}
    Pz.close()
    return out


def batched_legs(hq, count, pred, leaf=128, tol=1e-10):
    """count matrices of the batched generator in one spectral_projector_batched call: QDWH in FP64 and
    mixed precision, and Zolo-pd (one warmup and one timed call each); the errors of the mixed and
    Zolo-pd members against the FP64 ones."""
    import torch
    import workloads as wl
    mats = wl.batched_banded(count, seed=0)
    bs = [m.shape[1] - 1 for m in mats]
    mus = [hq.shift_for_count(m, bs[i], m.shape[0] // 2)[0] for i, m in enumerate(mats)]
    bands = [torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in mats]
    res = {"count": count, "sum_n": int(sum(m.shape[0] for m in mats))}
    keep = {}
    for prec in ("fp64", "mixed", "zolo"):
        kw = {"method": "zolo"} if prec == "zolo" else {"precision": prec}
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Ps, infos, st = hq.spectral_projector_batched(bands, bs, mus, leaf=leaf, tol=tol, predictor=pred, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if st != 0:
                raise RuntimeError(f"batched {prec}: status {st}")
            if rep == 0:
                for P in Ps:
                    P.close()
        print(f"# leg batched-{count} {prec}: {dt:.3f} s per batch", file=sys.stderr, flush=True)
        res[prec] = {"value": count / dt, "unit": "Π/s", "seconds": dt, "peak_bytes": infos[0]["peak_bytes"],
                     "redo_count": sum(i["redo_count"] for i in infos)}
        keep[prec] = Ps
    j = int(np.argmax([m.shape[0] for m in mats]))
    res["mixed"]["err_vs_fp64_2norm_largest_member"] = difference_norm(keep["mixed"][j], keep["fp64"][j],
                                                                       mats[j].shape[0])
    res["mixed"]["vs_fp64_batched"] = res["mixed"]["value"] / res["fp64"]["value"]
    res["zolo"]["err_vs_fp64_2norm_largest_member"] = difference_norm(keep["zolo"][j], keep["fp64"][j],
                                                                      mats[j].shape[0])
    res["zolo"]["vs_fp64_batched"] = res["zolo"]["value"] / res["fp64"]["value"]
    for Ps in keep.values():
        for P in Ps:
            P.close()
    return res


def main_batched(args, count, leaf=128, tol=1e-10):
    """One step = one spectral_projector_batched call over all `count` matrices."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    import paper_1608_01164_amd as hq
    import workloads as wl

    pred = _predictor(args.no_predictor)
    mats = wl.batched_banded(count, seed=0)
    bs = [m.shape[1] - 1 for m in mats]
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        mg = list(ex.map(lambda i: hq.shift_for_count(mats[i], bs[i], mats[i].shape[0] // 2), range(count)))
    mus = [x[0] for x in mg]
    bands = [torch.from_numpy(np.ascontiguousarray(m)).cuda() for m in mats]
    torch.cuda.synchronize()
    nsum = sum(m.shape[0] for m in mats)
    print(f"# workload {args.workload}: {count} matrices, sum n = {nsum}, b in [{min(bs)}, {max(bs)}], leaf={leaf}, "
          f"tol={tol}, min gap={min(x[1] for x in mg):.3e}", file=sys.stderr, flush=True)

    def step():
        Ps, infos, st = hq.spectral_projector_batched(bands, bs, mus, leaf=leaf, tol=tol, predictor=pred,
                                                      precision=args.precision, method=args.method)
        if st != 0:
            bad = [(i, mats[i].shape[0], bs[i], mg[i][1]) for i, P in enumerate(Ps) if P is None]
            print(f"# failed members (index, n, b, gap): {bad}; {hq.lib().hq_last_error().decode()}",
                  file=sys.stderr, flush=True)
            raise RuntimeError(f"batched solve: status {st}")
        return Ps, infos

    prof_w = None
    for i in range(args.warmup):
        last = i == args.warmup - 1 and not args.no_profile
        if last:
            hq.profile(True)
        Ps, infos = step()
        for P in Ps:
            P.close()
        if last:
            prof_w = hq.profile_read()
            hq.profile(False)
        for j, inf in enumerate(infos):
            print(f"#   member {j}: n={mats[j].shape[0]} b={bs[j]} K={inf['iters']} ranks/iter={inf['max_rank_iter']} "
                  f"redo={inf['redo_count']}", file=sys.stderr, flush=True)
        print(f"# warmup {i}: {infos[0]['seconds']:.3f} s, peak {infos[0]['peak_bytes'] / 2**30:.2f} GiB, "
              f"launches {infos[0]['launches']}", file=sys.stderr, flush=True)
    if not args.no_profile:
        hq.profile(True, classes=timed_classes(prof_w))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Ps = None
    for i in range(args.steps):
        if Ps is not None:
            for P in Ps:
                P.close()
        Ps, infos = step()
        print(f"# step {i}: {infos[0]['seconds']:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = hq.profile_read() if not args.no_profile else None
    mf = hq.binding.profile_mfma() if not args.no_profile else None
    if not args.no_profile:
        hq.profile(False)
    ms = 1e3 * (t1 - t0) / args.steps
    # at-any-size checks on the largest and the widest-band member
    chk = {}
    for j in sorted({int(np.argmax([m.shape[0] for m in mats])), int(np.argmax(bs))}):
        chk[f"member{j}_n{mats[j].shape[0]}_b{bs[j]}"] = properties(Ps[j], bands[j], mus[j])
    out = {
        "metric": METRIC, "value": count * args.steps / (t1 - t0), "unit": "Π/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32", "data": "synthetic",
        "config": {"workload": args.workload, "count": count, "sum_n": nsum, "leaf": leaf, "tol": tol,
                   "precision": args.precision, "method": args.method, "parallelism": "single-gpu, batched",
                   "capacities": "predictor" if pred is not None else "previous ranks"},
        "iters_max": max(i["iters"] for i in infos), "max_rank": max(i["max_rank"] for i in infos),
        "redo_count": sum(i["redo_count"] for i in infos), "launches": infos[0]["launches"],
        "peak_bytes": infos[0]["peak_bytes"], "checks": chk,
    }
    if prof is not None:
        out["roofline"] = roofline(prof, args.workload)
        out["mfma"] = mfma_util(mf, t1 - t0)
        out["kernels"] = kernel_table(prof_w if prof_w is not None else prof)
        out["kernels_source"] = "last warmup step, every kernel class timed" if prof_w is not None else "timed steps"
    print(json.dumps(out), flush=True)


# ---- the paper's timing and memory experiments (Sec. 6) on its synthetic test matrices ----------
# Matrices from the Sec. 6.1 construction: eigenvalues uniform in [-1, -gap] U [gap, 1] (half on each
# side, mu = 0) imposed on a b-banded matrix by plane rotations and bulge chasing.

# Memory of the HODLR projector reported in the paper's Table 2 (n = 16000, n_min = 250, eps = 1e-10,
# MATLAB on one Xeon core): MB for b = 1, 2, 4, 8, 16.
PAPER_TABLE2_MB = {1e-1: [55.72, 79.38, 127.04, 219.92, 395.91], 1e-4: [86.03, 129.71, 206.32, 340.88, 567.69]}


def _sec61(n, b, gap, seed=0):
    import workloads as wl
    return wl.prescribed_spectrum_band(wl.split_gap_spectrum(n, gap, seed), b)


def _time_projector(hq, ab, b, leaf, tol, reps=2, **kw):
    """Median seconds of `reps` projectors after one warmup, and the last call's info."""
    import torch
    band = torch.from_numpy(np.ascontiguousarray(ab)).cuda()
    ts = []
    info = None
    for i in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P, info = hq.spectral_projector(band, b, 0.0, leaf=leaf, tol=tol, **kw)
        torch.cuda.synchronize()
        if i > 0:
            ts.append(time.perf_counter() - t0)
        P.close()
    return float(np.median(ts)), info


def sweep_nmin(hq):
    """Example time_vs_nb_tridiag: time versus n_min for tridiagonal n = 50000."""
    for gap in (1e-1, 1e-4, 1e-6):
        ab = _sec61(50000, 1, gap)
        for leaf in (64, 128, 256, 512, 1024):
            t, info = _time_projector(hq, ab, 1, leaf, 1e-10)
            print(json.dumps({"sweep": "nmin", "n": 50000, "b": 1, "gap": gap, "n_min": leaf, "seconds": t,
                              "iters": info["iters"], "max_rank": info["max_rank"], "mb": info["bytes"] / 2**20}),
                  flush=True)


def sweep_memory(hq):
    """Example hodlrvshmatrix / Table 2: memory of the HODLR projector, n = 16000, n_min = 250, on the
    Sec. 6.1 matrices; and, for comparison, on banded matrices whose b bands are full (entries N(0,1),
    diagonal shift 4 i / n, mu at the middle of the spectrum, gap not controlled)."""
    import torch
    import workloads as wl
    for gap in (1e-1, 1e-4):
        for j, b in enumerate((1, 2, 4, 8, 16)):
            ab = _sec61(16000, b, gap)
            t, info = _time_projector(hq, ab, b, 250, 1e-10, reps=1)
            print(json.dumps({"sweep": "memory", "matrix": "sec6.1", "n": 16000, "b": b, "gap": gap, "n_min": 250,
                              "seconds": t, "mb": info["bytes"] / 2**20, "paper_mb": PAPER_TABLE2_MB[gap][j],
                              "max_rank": info["max_rank"], "iters": info["iters"]}), flush=True)
    for b in (1, 2, 4, 8, 16):
        ab = wl.banded_normal(16000, b, 0)
        mu, gap = hq.shift_for_count(ab, b, 8000)
        band = torch.from_numpy(np.ascontiguousarray(ab)).cuda()
        P, info = hq.spectral_projector(band, b, mu, leaf=250, tol=1e-10)
        P.close()
        print(json.dumps({"sweep": "memory", "matrix": "full-band normal", "n": 16000, "b": b, "gap": gap,
                          "n_min": 250, "seconds": info["seconds"], "mb": info["bytes"] / 2**20,
                          "max_rank": info["max_rank"], "iters": info["iters"]}), flush=True)


PAPER_TABLE2_H_MB = {1e-1: [95.16, 96.42, 106.54, 151.06, 291.85], 1e-4: [128.58, 160.56, 225.72, 352.54, 583.93]}


def sweep_hmatrix(hq):
    """Example hodlrvshmatrix / Table storage_spec: storage of the projector in HODLR and in the
    H-matrix format with the standard admissibility condition (Sec. 3.1.2), n = 16000, n_min = 250,
    eps = 1e-10, on the Sec. 6.1 matrices and on full-band normal ones.  Both counts use the actual
    ranks ((rows + cols) x rank per low-rank block, rows x cols per dense block)."""
    import torch
    import workloads as wl
    cases = [("sec6.1", gap, b, j) for gap in (1e-1, 1e-4) for j, b in enumerate((1, 2, 4, 8, 16))]
    cases += [("full-band normal", None, b, None) for b in (1, 2, 4, 8, 16)]
    for kind, gap, b, j in cases:
        if kind == "sec6.1":
            ab, mu = _sec61(16000, b, gap), 0.0
        else:
            ab = wl.banded_normal(16000, b, 0)
            mu, gap = hq.shift_for_count(ab, b, 8000)
        band = torch.from_numpy(np.ascontiguousarray(ab)).cuda()
        P, info = hq.spectral_projector(band, b, mu, leaf=250, tol=1e-10)
        t0 = time.perf_counter()
        H = hq.hodlr_to_hmatrix(P, 1e-10)
        dt = time.perf_counter() - t0
        sh = H.shape()
        row = {"sweep": "hmatrix", "matrix": kind, "n": 16000, "b": b, "gap": gap, "n_min": 250,
               "hodlr_mb": sh["hodlr_bytes"] / 2**20, "h_mb": sh["bytes"] / 2**20, "convert_s": dt,
               "low_rank_blocks": sh["low_rank_blocks"], "dense_blocks": sh["dense_blocks"],
               "h_max_rank": sh["max_rank"], "hodlr_max_rank": info["max_rank"]}
        if j is not None:
            row["paper_hodlr_mb"] = PAPER_TABLE2_MB[gap][j]
            row["paper_h_mb"] = PAPER_TABLE2_H_MB[gap][j]
        print(json.dumps(row), flush=True)
        H.close()
        P.close()


def sweep_scaling(hq):
    """Examples scaling_tridiag / band: time and memory versus n (gap 1e-6 tridiagonal, gap 1e-1 b = 4),
    and the 1D Laplacian (gap ~ 1/n)."""
    import workloads as wl
    for n in (4096, 8192, 16384, 32768, 65536, 131072):
        for kind, b in (("tridiag-gap1e-6", 1), ("band4-gap1e-1", 4), ("laplacian", 1)):
            if kind != "laplacian" and n > 32768:  # the O(n^2) construction of the test matrix
                continue
            ab = wl.laplacian(n) if kind == "laplacian" else _sec61(n, b, 1e-6 if b == 1 else 1e-1)
            t, info = _time_projector(hq, ab, b, 256 if b == 1 else 128, 1e-10, reps=1)
            print(json.dumps({"sweep": "scaling", "kind": kind, "n": n, "b": b, "seconds": t,
                              "mb": info["bytes"] / 2**20, "max_rank": info["max_rank"], "iters": info["iters"]}),
                  flush=True)


def sweep_breakeven(hq):
    """Breakeven versus a dense eigensolver (the paper: MATLAB eig on one core; here the GPU's dense
    symmetric eigensolver through torch.linalg.eigh, projector formed as V V^T), tridiagonal and b = 8;
    hQDWH and Zolo-pd."""
    import torch
    import workloads as wl
    for b, gap in ((1, 1e-1), (1, 1e-4), (8, 1e-1), (8, 1e-4)):
        for n in (1024, 2048, 4096, 8192, 16384):
            ab = _sec61(n, b, gap)
            t_h, info = _time_projector(hq, ab, b, 256 if b == 1 else 128, 1e-10)
            t_z, _ = _time_projector(hq, ab, b, 256 if b == 1 else 128, 1e-10, method="zolo")
            A = torch.from_numpy(wl.band_to_dense(ab)).cuda()
            ts = []
            for i in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lam, V = torch.linalg.eigh(A)
                Vn = V[:, : n // 2]
                Pi = Vn @ Vn.T
                torch.cuda.synchronize()
                if i > 0:
                    ts.append(time.perf_counter() - t0)
            del A, V, Vn, Pi
            print(json.dumps({"sweep": "breakeven", "n": n, "b": b, "gap": gap, "hqdwh_seconds": t_h,
                              "zolo_seconds": t_z, "dense_eigh_seconds": float(np.median(ts)),
                              "max_rank": info["max_rank"]}),
                  flush=True)


def sweep_solve(hq):
    """HODLR triangular solves (substitution with the H-Cholesky factor) against the products with the
    inverse factor, on diagonally dominant banded SPD matrices: factorisation and solve times, and
    the solution error against a dense solve where one fits."""
    import torch
    import workloads as wl
    for n, b, leaf in ((4096, 8, 128), (16384, 8, 128), (32768, 1, 256)):
        ab = np.array(wl.banded_normal(n, b, 17), dtype=np.float64)
        ab[:, 0] = np.abs(ab[:, 0]) + 2 * b * np.abs(ab).max() + 1.0
        H = hq.hodlr_build(torch.from_numpy(np.ascontiguousarray(ab)).cuda(), b, 0.0, 1.0, leaf=leaf)
        Bh = np.random.default_rng(3).standard_normal((8, n))
        B = torch.from_numpy(Bh).cuda()
        row = {"sweep": "solve", "n": n, "b": b, "leaf": leaf, "ncols": 8}
        xs = {}
        for method in ("substitution", "inverse"):
            X = torch.zeros_like(B)
            hq.cholesky_solve(H, B, X, tol=1e-12, method=method)  # warm
            tf, ts = hq.cholesky_solve(H, B, X, tol=1e-12, method=method)
            row[f"{method}_factor_s"] = tf
            row[f"{method}_solve_s"] = ts
            xs[method] = X.cpu().numpy()
        row["max_diff"] = float(np.abs(xs["substitution"] - xs["inverse"]).max())
        if n <= 4096:
            ref = np.linalg.solve(wl.band_to_dense(ab), Bh.T).T
            row["err_substitution"] = float(np.abs(xs["substitution"] - ref).max() / np.abs(ref).max())
            row["err_inverse"] = float(np.abs(xs["inverse"] - ref).max() / np.abs(ref).max())
        H.close()
        print(json.dumps(row), flush=True)


SWEEPS = {"nmin": sweep_nmin, "memory": sweep_memory, "scaling": sweep_scaling, "breakeven": sweep_breakeven,
          "hmatrix": sweep_hmatrix, "solve": sweep_solve}


if __name__ == "__main__":
    main()
