"""Each building block of the HIP path through the C ABI, against numpy FP64 references."""
import numpy as np
import pytest

import paper_1608_01164_amd as hq
from oracle import hodlr as oh
from tests.gpu_util import dev, empty, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,k,opA,opB", [
    (1, 1, 1, 0, 0), (64, 64, 16, 0, 0), (65, 63, 17, 0, 1), (130, 7, 300, 1, 0), (33, 129, 5, 1, 1),
    (1000, 40, 40, 0, 0), (40, 40, 3000, 1, 0), (7, 3, 0, 0, 0),
    # split K (k >= 512): 2, 3 and 32 ranges, ragged tiles
    (70, 150, 513, 1, 0), (150, 150, 1023, 1, 0), (129, 65, 8192, 1, 1), (64, 64, 8200, 0, 0)])
def test_gemm(m, n, k, opA, opB):
    rng = np.random.default_rng(m * 7 + n)
    A = rng.standard_normal((k, m) if opA else (m, k))
    B = rng.standard_normal((n, k) if opB else (k, n))
    if k == 0:  # keep non-null device buffers
        A = np.zeros((m, 1))
        B = np.zeros((1, n))
    C = rng.standard_normal((m, n))
    dA, dB, dC = dev(A), dev(B), dev(C)
    hq.test_gemm(dA, dB, dC, m, n, k, A.shape[0], B.shape[0], m, opA, opB, 1.5, -0.5)
    ref = (1.5 * (A.T if opA else A) @ (B.T if opB else B) if k else 0.0) - 0.5 * C
    got = host(dC, m, n)
    assert np.abs(got - ref).max() <= 1e-13 * max(1.0, k) ** 0.5 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("m,n,k,opA,opB", [
    (16, 16, 16, 0, 0), (64, 64, 16, 0, 0), (65, 63, 17, 0, 1), (130, 7, 300, 1, 0), (33, 129, 5, 1, 1),
    (1000, 40, 40, 0, 0), (40, 40, 3000, 1, 0)])
def test_gemm_fp32(m, n, k, opA, opB):
    """FP32 MFMA variant: operands rounded to FP32, FP32 accumulation.  The identity product
    pins the placement of every output row; the random product is checked within FP32 rounding."""
    if (m, n, k) == (16, 16, 16):
        A = np.eye(16)
        B = np.arange(256, dtype=np.float64).reshape(16, 16)  # exact in FP32
        dC = empty(16, 16)
        hq.test_gemm(dev(A), dev(B), dC, 16, 16, 16, 16, 16, 16, 0, 0, 1.0, 0.0, fp32=True)
        assert np.array_equal(host(dC, 16, 16), B)
        return
    rng = np.random.default_rng(m * 7 + n + 1)
    A = rng.standard_normal((k, m) if opA else (m, k))
    B = rng.standard_normal((n, k) if opB else (k, n))
    C = rng.standard_normal((m, n))
    dC = dev(C)
    hq.test_gemm(dev(A), dev(B), dC, m, n, k, A.shape[0], B.shape[0], m, opA, opB, 1.5, -0.5, fp32=True)
    Af, Bf = (A.T if opA else A), (B.T if opB else B)
    ref = 1.5 * Af @ Bf - 0.5 * C
    bound = 1.5 * np.abs(Af) @ np.abs(Bf) * 4 * k * np.finfo(np.float32).eps
    assert (np.abs(host(dC, m, n) - ref) <= bound + 1e-12).all()


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("m,n,k,opA,opB", [
    (1, 1, 1, 0, 0), (16, 16, 4, 0, 1), (65, 63, 17, 0, 1), (130, 7, 300, 1, 0), (33, 129, 5, 1, 1),
    (128, 128, 128, 0, 1), (1000, 40, 65, 1, 1), (300, 300, 511, 0, 0), (7, 3, 0, 0, 0)])
def test_gemm_small_and_tiled_kernels_agree(m, n, k, opA, opB, fp32):
    """The 32 x 32 register-staged kernel (launches of few tiles) and the 64 x 64 LDS-staged one issue
    the same MFMAs in the same K order: forcing either through the tuning table gives the same C bit
    for bit, and both match numpy."""
    rng = np.random.default_rng(m * 11 + n * 3 + k)
    A = rng.standard_normal((max(k, 1), m) if opA else (m, max(k, 1)))
    B = rng.standard_normal((n, max(k, 1)) if opB else (max(k, 1), n))
    C = rng.standard_normal((m, n))
    out = []
    for small in (0, 1 << 20):
        old = hq.set_tuning(gemm_small_tiles=small)
        try:
            dC = dev(C)
            hq.test_gemm(dev(A), dev(B), dC, m, n, k, A.shape[0], B.shape[0], m, opA, opB, 1.5, -0.5, fp32=fp32)
            out.append(host(dC, m, n))
        finally:
            hq.set_tuning(gemm_small_tiles=old["gemm_small_tiles"])
    assert np.array_equal(out[0], out[1])
    Af = (A.T if opA else A)[:, :k]
    Bf = (B.T if opB else B)[:k, :]
    ref = 1.5 * Af @ Bf - 0.5 * C
    eps = np.finfo(np.float32 if fp32 else np.float64).eps
    bound = 1.5 * np.abs(Af) @ np.abs(Bf) * 4 * max(k, 1) * eps
    assert (np.abs(out[0] - ref) <= bound + 1e-12).all()


@pytest.mark.parametrize("rows,r", [(300, 20), (3000, 40), (700, 200), (5000, 150), (128, 100), (200, 90)])
def test_qr_r_fp32(rows, r):
    rng = np.random.default_rng(rows + r + 1)
    M = rng.standard_normal((rows, r)) * np.logspace(0, -3, r)[None, :]
    dR = empty(r, r)
    hq.test_qr_r(dev(M), rows, r, rows, dR, fp32=True)
    R = host(dR, r, r)
    assert np.abs(np.tril(R, -1)).max() == 0.0
    Rn = np.linalg.qr(M, mode="r")
    # backward stable in FP32: R^T R reproduces M^T M to O(u32) relative to ||M||^2
    assert np.abs(R.T @ R - Rn.T @ Rn).max() <= 50 * np.finfo(np.float32).eps * np.linalg.norm(M, 2) ** 2


# tiles of at most 128 rows and 256 columns, or 256 rows and 128 columns, are factored in registers;
# a stack with no more rows than columns is passed on as its own factor (M = I M)
# several row tiles: the tree steps combine two stacked triangles (structured for r <= 192, a ragged
# last tile giving a trapezoid below), dense above
@pytest.mark.parametrize("rows,r", [(1, 1), (5, 9), (64, 64), (300, 20), (2000, 37), (9000, 64), (700, 200),
                                    (128, 200), (100, 130), (128, 127), (128, 60), (129, 60), (200, 100),
                                    (256, 128), (250, 129), (3000, 150), (4100, 190), (2500, 100), (5000, 131),
                                    (1100, 192), (2100, 200), (8300, 70), (2150, 120)])
def test_qr_r(rows, r):
    rng = np.random.default_rng(rows + r)
    M = rng.standard_normal((rows, r)) * np.logspace(0, -12, r)[None, :]
    dM = dev(M)
    dR = empty(r, r)
    hq.test_qr_r(dM, rows, r, rows, dR)
    R = host(dR, r, r)
    if rows <= r:
        assert np.array_equal(R[:rows], M) and not R[rows:].any()
        return
    assert np.abs(np.tril(R, -1)).max() == 0.0
    Rn = np.linalg.qr(M, mode="r")
    kk = min(rows, r)
    # R is unique up to row signs
    assert np.abs(np.abs(R[:kk]) - np.abs(Rn[:kk])).max() < 1e-12 * np.abs(Rn).max()
    if rows < r:
        assert np.abs(R[kk:]).max() == 0.0


@pytest.mark.parametrize("m,n,r,decay", [(300, 200, 40, 0.6), (1200, 900, 90, 0.8), (64, 64, 64, 0.5)])
def test_recompress_fp32(m, n, r, decay):
    """FP32 recompression: the error is at the FP32 truncation level max(tol, 4 u32 sqrt(rows)
    sigma_1) (times a modest factor for the FP32 arithmetic), and no kept direction is spurious."""
    rng = np.random.default_rng(m + n + r + 5)
    s = decay ** np.arange(r)
    Uq, _ = np.linalg.qr(rng.standard_normal((m, r)))
    Vq, _ = np.linalg.qr(rng.standard_normal((n, r)))
    Us = np.hstack([Uq * s, 0.5 * Uq[:, : r // 2] * s[: r // 2]])
    Vs = np.hstack([Vq, Vq[:, : r // 2]])
    rr = Us.shape[1]
    M = Us @ Vs.T
    U, V = empty(m, rr), empty(n, rr)
    k = hq.test_recompress(dev(Us), m, dev(Vs), n, rr, 1e-10, rr, U, V, fp32=True)
    sv = np.linalg.svd(M, compute_uv=False)
    eff = 4 * np.finfo(np.float32).eps / 2 * np.sqrt(max(m, n)) * sv[0]  # u32 = eps / 2
    assert int(np.sum(sv > 4 * eff)) <= k <= int(np.sum(sv > eff / 4))
    Uh, Vh = host(U, m, k), host(V, n, k)
    assert np.linalg.norm(Uh @ Vh.T - M, 2) <= 4 * eff


@pytest.mark.parametrize("rows,r", [(300, 20), (3000, 40), (120, 90), (200, 60), (3000, 150), (2200, 100)])
def test_qr_r_columns_near_underflow(rows, r):
    """Columns scaled into the range where squared norms are denormal or underflow: the
    triangular factor stays finite and matches LAPACK's column by column (relative to each
    column's own size)."""
    rng = np.random.default_rng(rows * r)
    scales = np.array([10.0 ** -(140 + 20 * (c % 9)) if c % 3 else 1.0 for c in range(r)])
    M = rng.standard_normal((rows, r)) * scales[None, :]
    dR = empty(r, r)
    hq.test_qr_r(dev(M), rows, r, rows, dR)
    R = host(dR, r, r)
    assert np.isfinite(R).all()
    Rn = np.linalg.qr(M, mode="r")
    kk = min(rows, r)
    for c in range(r):
        ref = np.abs(M[:, c]).max()  # a plain 2-norm of such a column underflows
        assert np.abs(np.abs(R[:kk, c]) - np.abs(Rn[:kk, c])).max() <= 1e-12 * ref * np.sqrt(rows)


# stacked widths 1.5 r: cores of up to 128, 256 and 512 columns take the register paths (16-lane
# groups, then 32-lane groups), wider ones the looped path; the two 256-column cases keep whole
# 256-row column segments in LDS (rank about 31: C and J there; about 60: C there, J global)
@pytest.mark.parametrize("m,n,r,decay", [(50, 60, 10, 1.0), (300, 200, 40, 0.6), (1200, 900, 90, 0.8),
                                         (64, 64, 64, 0.5), (10, 400, 30, 0.3), (600, 700, 180, 0.85),
                                         (1500, 1200, 200, 0.88), (2000, 2000, 300, 0.92), (2000, 1800, 360, 0.9),
                                         (600, 500, 171, 0.45), (1500, 1200, 171, 0.656),
                                         (800, 700, 140, 0.72), (900, 800, 200, 0.6),
                                         # stacks wider than the block: the core runs on its leading square
                                         (120, 110, 200, 0.8), (200, 150, 300, 0.7)])
def test_recompress(m, n, r, decay):
    rng = np.random.default_rng(m + n + r)
    s = decay ** np.arange(r)
    Uq, _ = np.linalg.qr(rng.standard_normal((m, r)))
    Vq, _ = np.linalg.qr(rng.standard_normal((n, r)))
    kk = min(m, n, r)
    Us = Uq[:, :kk] * s[:kk]
    Vs = Vq[:, :kk]
    # stack redundant copies so that recompression has something to remove
    Us2 = np.hstack([Us, 0.5 * Us[:, : kk // 2]])
    Vs2 = np.hstack([Vs, Vs[:, : kk // 2]])
    rr = Us2.shape[1]
    M = Us2 @ Vs2.T
    tol = 1e-10
    U, V = empty(m, rr), empty(n, rr)
    k = hq.test_recompress(dev(Us2), m, dev(Vs2), n, rr, tol, rr, U, V)
    sv = np.linalg.svd(M, compute_uv=False)
    assert k == int(np.sum(sv > tol))
    Uh, Vh = host(U, m, k), host(V, n, k)
    assert np.linalg.norm(Uh @ Vh.T - M, 2) <= tol + 1e-13 * sv[0]
    # V is orthonormal where it matters: the Schur update U (V^T V) U^T equals U U^T to rounding
    assert np.abs(Uh @ (Vh.T @ Vh - np.eye(k)) @ Uh.T).max() < 1e-13 * max(1.0, sv[0] ** 2)


@pytest.mark.parametrize("m,n,r", [(40, 50, 12), (600, 500, 200)])
def test_recompress_nonfinite_is_reported(m, n, r):
    """Regression: NaN stacks used to leave the core SVD's pivot search without a candidate; the
    kernel now stops and the call reports non-finite values instead of touching memory."""
    rng = np.random.default_rng(7)
    Us = rng.standard_normal((m, r))
    Vs = rng.standard_normal((n, r))
    Us[:, :] = np.nan
    U, V = empty(m, r), empty(n, r)
    with pytest.raises(hq.HQError) as e:
        hq.test_recompress(dev(Us), m, dev(Vs), n, r, 1e-10, r, U, V)
    assert e.value.status == 5
    # the library stays usable afterwards
    Us = rng.standard_normal((m, 3)) @ rng.standard_normal((3, r))
    k = hq.test_recompress(dev(Us), m, dev(Vs), n, r, 1e-10, r, U, V)
    assert k == 3


def _kernel_matrix(n, seed):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(0, 1, n))
    return 1.0 / (1.0 + 30 * np.abs(x[:, None] - x[None, :])) + 0.1 * np.eye(n)


@pytest.mark.parametrize("n,leaf", [(100, 16), (257, 32), (512, 64)])
def test_from_dense_roundtrip(n, leaf):
    K = _kernel_matrix(n, n)
    H = hq.test_from_dense(dev(K), n, leaf, 1e-12, 128)
    D = H.to_dense().cpu().numpy()
    assert np.abs(D - K).max() < 1e-10
    E = H.export()
    assert np.abs(oh.to_dense(E) - K).max() < 1e-10
    X = np.random.default_rng(1).standard_normal((n, 5))
    import torch
    Y = H.apply(torch.from_numpy(X).cuda()).cpu().numpy()
    assert np.abs(Y - K @ X).max() < 1e-9


@pytest.mark.parametrize("n,leaf,tA,tB", [(200, 25, 0, 0), (333, 40, 1, 0), (256, 32, 0, 1), (512, 64, 1, 1)])
def test_product(n, leaf, tA, tB):
    A = _kernel_matrix(n, 1)
    B = _kernel_matrix(n, 2) + 0.3 * np.triu(_kernel_matrix(n, 3), 1)
    D = _kernel_matrix(n, 4)
    tol = 1e-11
    hA = hq.test_from_dense(dev(A), n, leaf, 1e-13, 200)
    hB = hq.test_from_dense(dev(B), n, leaf, 1e-13, 200)
    hD = hq.test_from_dense(dev(D), n, leaf, 1e-13, 200)
    C = hq.test_product(hA, tA, hB, tB, 0.7, hD, 0, -1.3, 0, 200, tol)
    ref = 0.7 * (A.T if tA else A) @ (B.T if tB else B) - 1.3 * D
    got = C.to_dense().cpu().numpy()
    assert np.abs(got - ref).max() < 1e-9
    # symmetric Z = I + c X^T X in lower storage
    Z = hq.test_product(hA, 1, hA, 0, 2.0, None, 1, 1.0, 1, 200, tol)
    Zd = oh.to_dense(Z.export())
    Zref = np.eye(n) + 2.0 * A.T @ A
    assert np.abs(np.tril(Zd) - np.tril(Zref)).max() < 1e-9


# leaves up to 128 rows: one fused kernel; 129..256: 2 x 2 split around it; above: the looped kernels
@pytest.mark.parametrize("n,leaf", [(64, 64), (200, 25), (300, 37), (512, 64), (5, 5), (128, 128), (129, 129),
                                    (256, 256), (400, 200), (320, 160), (300, 300)])
def test_cholesky_inverse(n, leaf):
    A = _kernel_matrix(n, 5)
    Z = np.eye(n) + 3.0 * A.T @ A
    hZ = hq.test_from_dense(dev(Z), n, leaf, 1e-13, 200)
    Li = hq.test_cholesky_inverse(hZ, 200, 1e-12)
    G = oh.to_dense(Li.export())
    Lref = np.linalg.cholesky(Z)
    assert np.abs(np.triu(G, 1)).max() == 0.0
    assert np.abs(G @ Z @ G.T - np.eye(n)).max() < 1e-9
    assert np.abs(G - np.linalg.inv(Lref)).max() < 1e-9


@pytest.mark.parametrize("n,leaf,row", [(64, 64, 0), (128, 128, 93), (126, 126, 125), (300, 37, 41),
                                        (200, 200, 50), (200, 200, 150), (255, 255, 254)])
def test_cholesky_inverse_indefinite_is_reported(n, leaf, row):
    """A leaf whose Schur complement loses positive definiteness (a negative eigenvalue planted in
    the coupling of row `row`) reports status 2; padded rows of a ragged leaf never do."""
    A = _kernel_matrix(n, 5)
    Z = np.eye(n) + 0.1 * A.T @ A
    d0 = Z[row, row]
    Z[row, row] = -1.0
    hZ = hq.test_from_dense(dev(Z), n, leaf, 1e-13, 200)
    with pytest.raises(hq.HQError) as e:
        hq.test_cholesky_inverse(hZ, 200, 1e-12)
    assert e.value.status == 2
    Z[row, row] = d0 + 1.0  # the library stays usable, and the same matrix made definite factors
    hZ = hq.test_from_dense(dev(Z), n, leaf, 1e-13, 200)
    G = oh.to_dense(hq.test_cholesky_inverse(hZ, 200, 1e-12).export())
    assert np.abs(G @ Z @ G.T - np.eye(n)).max() < 1e-9


@pytest.mark.parametrize("n,b,leaf", [(64, 1, 8), (300, 1, 64), (257, 5, 40), (512, 8, 64)])
def test_q_factors_device(n, b, leaf):
    import workloads as w
    from oracle import givens_qr as g
    ab = w.tridiag_uniform(n, 2) if b == 1 else w.banded_normal(n, b, 2)
    A = w.band_to_dense(ab)
    Q, R, rots = g.fast_qr(1.7 * (A - 0.05 * np.eye(n)), b)
    h1, h2, nr = hq.test_q_factors(ab, b, 0.05, 1.7, leaf)
    assert nr == len(rots)
    assert np.abs(oh.to_dense(h1.export()) - Q[:n, :n]).max() < 1e-13
    assert np.abs(h2.to_dense().cpu().numpy() - Q[n:, :n]).max() < 1e-13


@pytest.mark.parametrize("n,b,leaf", [(1000, 3, 64), (777, 1, 32), (2048, 8, 128), (300, 2, 300)])
def test_cholesky_solve_substitution_and_inverse(n, b, leaf):
    """HODLR triangular solves by substitution with the H-Cholesky factor, and the route through the
    inverse factor the iteration takes, both solve a symmetric positive definite banded system to the
    truncation level and agree with each other; B is left as it was."""
    import torch
    import workloads as w
    ab = np.array(w.banded_normal(n, b, 17), dtype=np.float64)
    ab[:, 0] = np.abs(ab[:, 0]) + 2 * b * np.abs(ab).max() + 1.0  # diagonally dominant: SPD
    A = w.band_to_dense(ab)
    H = hq.hodlr_build(torch.from_numpy(np.ascontiguousarray(ab)).cuda(), b, 0.0, 1.0, leaf=leaf)
    Bh = np.random.default_rng(3).standard_normal((5, n))  # five right-hand sides (n x 5 column-major)
    B = torch.from_numpy(Bh).cuda()
    ref = np.linalg.solve(A, Bh.T)
    out = {}
    for method in ("substitution", "inverse"):
        X = torch.zeros_like(B)
        tf, ts = hq.cholesky_solve(H, B, X, tol=1e-13, method=method)
        Xh = X.cpu().numpy().T
        assert np.abs(Xh - ref).max() <= 1e-9 * np.abs(ref).max(), method
        assert np.array_equal(B.cpu().numpy(), Bh)
        assert tf > 0 and ts > 0
        out[method] = Xh
    assert np.abs(out["substitution"] - out["inverse"]).max() <= 1e-9 * np.abs(ref).max()
    H.close()
