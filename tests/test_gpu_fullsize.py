"""Parity at the benchmark's full sizes, in the configuration bench.py times (trained rank predictor,
library defaults, band resident on the device).

Banded n = 16384, b = 8 (the benchmark's workload), FP64 and mixed: the oracle computes all n
eigenpairs (bisection + inverse iteration), so D = P - Pi_o is measured as a norm:
  * ||D||_2 by Lanczos on x -> P x - V_nu (V_nu^T x) (P applied on the device, V_nu the oracle's
    eigenvectors below mu, kept factored);
  * ||D||_F = (sum_i ||D v_i||^2)^(1/2) over the whole orthonormal eigenbasis, where D v_i = P v_i - v_i
    below mu and P v_i above: a certified upper bound of ||D||_2 (up to the basis' orthonormality,
    checked to 1e-12).
The larger workloads (n = 32768, 100000, the batched members) keep the oracle to sampled outputs:
eigenpairs for the eight eigenvalues on each side of mu (where the projector is hardest) and eight
spread over the spectrum; Pi v_i is v_i or 0, so ||P v_i - Pi v_i||_2 <= ||P - Pi||_2 checks the gate
direction by direction.  Properties that hold at any size are checked on random vectors: with
D = P - Pi, P^2 - P = Pi D + D Pi + D^2 - D and A P - P A = A D - D A, so ||P^2 - P|| <= 4 ||D|| and
||A P - P A|| <= 2 ||A|| ||D||.
"""
import time

import numpy as np
import pytest

import paper_1608_01164_amd as hq
import workloads as w
from oracle import eig, norms
from tests.mixed_model import TOL_AFTER_FP32, bound_from_info

pytestmark = pytest.mark.gpu

GATE = 1e-8  # ||P - Pi||_2 in FP64 mode


def _sample(ab, nu, rng):
    n = ab.shape[0]
    near = list(range(max(1, nu - 7), min(n, nu + 8) + 1))
    spread = sorted(set(int(k) for k in rng.integers(1, n + 1, size=8)) - set(near))
    idx = sorted(set(near) | set(spread))
    lam = np.concatenate([eig.eigenvalues(ab, k, k) for k in idx])
    return np.array(idx), lam, eig.eigenvectors(ab, lam)


def _band_matvec_dev(band, X):
    n, ld = band.shape
    Y = band[:, 0:1] * X
    for i in range(1, ld):
        c = band[: n - i, i: i + 1]
        Y[i:] += c * X[: n - i]
        Y[: n - i] += c * X[i:]
    return Y


def _properties(P, band, mu, seed=0):
    import torch
    n = band.shape[0]
    g = torch.Generator(device="cuda").manual_seed(seed)
    X = torch.randn((n, 4), generator=g, dtype=torch.float64, device="cuda")
    PX = P.apply(X)
    PPX = P.apply(PX.contiguous())
    AX = _band_matvec_dev(band, X)
    APX = _band_matvec_dev(band, PX)
    PAX = P.apply(AX.contiguous())
    QX, AQX = X - PX, AX - APX
    return {
        "idem": float((PPX - PX).norm() / X.norm()),
        "comm": float((APX - PAX).norm() / X.norm()),
        "neg": float(((PX * (APX - mu * PX)).sum(0) / (PX * PX).sum(0)).max()),
        "pos": float(((QX * (AQX - mu * QX)).sum(0) / (QX * QX).sum(0)).min()),
    }


def _last_tol(info, tol):
    """Truncation tolerance of the last iteration: FP64 iterations after FP32 ones (mixed mode) truncate
    at max(tol, TOL_AFTER_FP32)."""
    return max(tol, TOL_AFTER_FP32) if any(info["fp32_iter"]) else tol


def _check_properties(name, ab, P, band, mu, bound, levels, tol):
    pr = _properties(P, band, mu)
    anorm = float(np.abs(ab).sum(1).max()) * 2  # ||A||_inf of the symmetric matrix (band stores one triangle)
    # The last iteration and the symmetrisation run in FP64 in every mode and drive the eigenvalues to
    # 0 and 1 up to the truncations of the final iterate (at most tol per level), whatever the
    # rotation of the invariant subspace: ||P^2 - P|| <= levels * tol as well as <= 4 ||D||.
    idem_bound = min(4 * bound, levels * tol)
    print(f"    {name}: idem {pr['idem']:.2e} (<= {idem_bound:.1e})  comm {pr['comm']:.2e} "
          f"(<= {2 * anorm * bound:.1e})  rayleigh {pr['neg']:.3f} / {pr['pos']:.3f}", flush=True)
    assert pr["idem"] <= idem_bound
    assert pr["comm"] <= 2 * anorm * bound
    assert pr["neg"] < 0 < pr["pos"]


@pytest.fixture(scope="module")
def default_predictor():
    from paper_1608_01164_amd import predictor as hp
    return hp.load()


@pytest.fixture(scope="module")
def banded16384():
    """The oracle's complete eigen-decomposition of the benchmark's matrix (n = 16384, b = 8)."""
    import torch
    ab = w.banded_normal(16384, 8, 0)
    n = ab.shape[0]
    t0 = time.perf_counter()
    lam = eig.eigenvalues(ab, 1, n)
    V = eig.eigenvectors(ab, lam)
    Vd = torch.from_numpy(np.ascontiguousarray(V.T)).cuda().T  # column-major view on the device
    G = Vd.T @ Vd
    orth = float((G - torch.eye(n, dtype=torch.float64, device="cuda")).abs().max())
    del G
    print(f"\noracle: {n} eigenpairs in {time.perf_counter() - t0:.1f} s on {eig.num_threads()} threads, "
          f"max |V^T V - I| = {orth:.2e}", flush=True)
    assert orth <= 1e-12
    return ab, lam, V, Vd


def _method_opts(precision):
    """'zolo' selects Zolo-pd (FP64); otherwise QDWH in that precision."""
    return {"method": "zolo"} if precision == "zolo" else {"precision": precision}


@pytest.mark.parametrize("precision", ["fp64", "mixed", "zolo"])
def test_banded16384_norm_parity(default_predictor, banded16384, precision):
    """||P - Pi_o||_2 (Lanczos) and the certified ||P - Pi_o||_F on the benchmark's workload (QDWH in
    FP64 and mixed precision, and Zolo-pd)."""
    import torch
    ab, lam, V, Vd = banded16384
    n = ab.shape[0]
    nu = n // 2
    mu = 0.5 * (lam[nu - 1] + lam[nu])
    band = torch.from_numpy(np.ascontiguousarray(ab)).cuda()
    P, info = hq.spectral_projector(band, 8, mu, leaf=128, tol=1e-10, predictor=default_predictor,
                                    **_method_opts(precision))
    bound = GATE if precision != "mixed" else bound_from_info(n, info)
    # certified Frobenius norm over the whole eigenbasis
    ss = 0.0
    for c0 in range(0, n, 2048):
        blk = Vd[:, c0:c0 + 2048].contiguous()
        D = P.apply(blk)
        if c0 < nu:
            D[:, : min(2048, nu - c0)] -= blk[:, : min(2048, nu - c0)]
        ss += float((D * D).sum())
        del D, blk
    frob = ss ** 0.5
    Vb = V[:, :nu]

    def op(x):
        y = P.apply(torch.from_numpy(x.reshape(n, 1)).cuda()).cpu().numpy().ravel()
        return y - Vb @ (Vb.T @ x)

    two = norms.lanczos_norm(op, n, steps=60)
    print(f"banded-n16384-b8 {precision}: gap={lam[nu] - lam[nu - 1]:.3e} K={info['iters']} "
          f"fp32 iterations={info['fp32_iter']} maxrank={info['max_rank']} redo={info['redo_count']} "
          f"t={info['seconds']:.2f}s | ||P-Pi||_2 (Lanczos) {two:.3e}  ||P-Pi||_F {frob:.3e}  bound {bound:.2e}",
          flush=True)
    assert two <= bound
    if precision != "mixed":
        assert frob <= 10 * GATE
    _check_properties("banded-n16384-b8", ab, P, band, mu, bound, info["levels"], _last_tol(info, 1e-10))
    P.close()


FULL = [
    # name, band maker, b, leaf, tol, precision, bound on ||(P - Pi) v||_2 (None: the stated mixed bound)
    ("metallic-n32768", lambda: w.tridiag_metallic(32768, 0), 1, 256, 1e-10, "fp64", GATE),
    ("metallic-n32768-mixed", lambda: w.tridiag_metallic(32768, 0), 1, 256, 1e-10, "mixed", None),
    ("tridiag-n100000-tol1e-8", lambda: w.tridiag_uniform(100000, 0), 1, 256, 1e-8, "fp64", GATE),
    ("tridiag-n100000-tol1e-8-mixed", lambda: w.tridiag_uniform(100000, 0), 1, 256, 1e-8, "mixed", None),
    ("metallic-n32768-zolo", lambda: w.tridiag_metallic(32768, 0), 1, 256, 1e-10, "zolo", GATE),
]


@pytest.mark.parametrize("name,maker,b,leaf,tol,precision,bound", FULL, ids=[c[0] for c in FULL])
def test_full_size_sampled_parity(default_predictor, name, maker, b, leaf, tol, precision, bound):
    import torch
    ab = maker()
    n = ab.shape[0]
    nu = n // 2
    mu, gap, _ = eig.midpoint_shift(ab, nu)
    idx, lam, V = _sample(ab, nu, np.random.default_rng(n))
    band = torch.from_numpy(np.ascontiguousarray(ab)).cuda()
    P, info = hq.spectral_projector(band, b, mu, leaf=leaf, tol=tol, predictor=default_predictor,
                                    **_method_opts(precision))
    PV = P.apply(torch.from_numpy(np.ascontiguousarray(V)).cuda()).cpu().numpy()
    below = lam < mu
    assert below.sum() == np.count_nonzero(idx <= nu)
    err = np.linalg.norm(PV - V * below[None, :], axis=0)
    if bound is None:
        bound = bound_from_info(n, info)
    near = np.abs(idx - nu - 0.5) < 8
    print(f"{name}: n={n} b={b} gap={gap:.3e} K={info['iters']} fp32 iterations={info['fp32_iter']} "
          f"maxrank={info['max_rank']} redo={info['redo_count']} t={info['seconds']:.2f}s | max ||(P-Pi)v|| next "
          f"to mu {err[near].max():.3e}, elsewhere {err[~near].max() if (~near).any() else 0:.3e} | bound {bound:.2e}",
          flush=True)
    assert err.max() <= bound
    _check_properties(name, ab, P, band, mu, bound, info["levels"], _last_tol(info, tol))
    P.close()


def test_full_size_batched_members(default_predictor):
    """The batched workload's generator (n_i ~ U{2048..16384}, b_i ~ U{1..16}): 16 members in one
    batched call, the largest n and the widest band among the first 64 included; every member's
    projector checked on sampled eigenvectors next to its mu."""
    import torch
    rs = np.random.default_rng(0)
    ns = rs.integers(2048, 16385, size=64)
    bs = rs.integers(1, 17, size=64)
    pick = sorted(set(range(14)) | {int(np.argmax(ns)), int(np.argmax(bs))})[:16]
    mats = [w.banded_normal(int(ns[i]), int(bs[i]), rng=np.random.default_rng([0, i])) for i in pick]
    bws = [int(bs[i]) for i in pick]
    mus, samples = [], []
    for ab in mats:
        n = ab.shape[0]
        mu, _, _ = eig.midpoint_shift(ab, n // 2)
        mus.append(mu)
        lam = eig.eigenvalues(ab, n // 2 - 3, n // 2 + 4)
        samples.append((lam, eig.eigenvectors(ab, lam)))
    bands = [torch.from_numpy(np.ascontiguousarray(ab)).cuda() for ab in mats]
    Ps, infos, st = hq.spectral_projector_batched(bands, bws, mus, leaf=128, tol=1e-10, predictor=default_predictor)
    assert st == 0
    worst = 0.0
    for j, (P, (lam, V)) in enumerate(zip(Ps, samples)):
        PV = P.apply(torch.from_numpy(np.ascontiguousarray(V)).cuda()).cpu().numpy()
        err = np.linalg.norm(PV - V * (lam < mus[j])[None, :], axis=0).max()
        worst = max(worst, err)
        assert err <= GATE, (pick[j], mats[j].shape[0], bws[j], err)
        P.close()
    print(f"batched 16 members (sum n = {sum(m.shape[0] for m in mats)}): worst sampled ||(P-Pi)v|| {worst:.3e}, "
          f"{infos[0]['seconds']:.2f}s")
