"""The allocation-free apply (apply_projector_noalloc) against apply_projector on the same projector:
two calls in a row, the second with a smaller input, and a request above the static workspace
maximum rejected before anything runs."""
import pytest

import paper_1608_01164_amd as hq
import workloads as w

pytestmark = pytest.mark.gpu


def _projector(n, b, leaf, seed):
    import torch
    ab = w.banded_normal(n, b, seed)
    mu, _ = hq.shift_for_count(ab, b, n // 2)
    P, _ = hq.spectral_projector(torch.from_numpy(ab).cuda(), b, mu, leaf=leaf, tol=1e-10)
    return P


def _check_against_apply(P, k, seed):
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    Xt = torch.randn((k, P.n), generator=g, dtype=torch.float64, device="cuda")
    ref = P.apply(Xt.t()).t().contiguous()           # apply_projector, (k, n) rows = columns of Y
    Yt = torch.full_like(Xt, float("nan"))
    P.apply_noalloc(Xt, Yt)
    torch.cuda.synchronize()
    scale = float(ref.abs().max())
    err = float((Yt - ref).abs().max())
    print(f"noalloc n={P.n} k={k}: max |Y - Y_apply| = {err:.3e} (scale {scale:.3e}), "
          f"bitwise {bool(torch.equal(Yt, ref))}", flush=True)
    # same kernels, same task lists, same reduction orders: the bar is the FP64 rounding of one apply
    assert err <= 1e-13 * max(scale, 1.0)


def test_noalloc_apply_two_calls_second_smaller():
    P = _projector(2048, 8, 128, 3)
    _check_against_apply(P, 24, 1)
    P2 = _projector(700, 3, 64, 4)        # smaller matrix and fewer columns on the second call
    _check_against_apply(P2, 5, 2)
    _check_against_apply(P, 3, 5)         # back to the first handle: stale workspace contents unused
    P.close()
    P2.close()


def test_noalloc_apply_rejects_beyond_static_maximum():
    import torch
    P = _projector(2048, 8, 128, 3)
    cap = hq.lib().apply_projector_noalloc_max_bytes()
    assert cap == 64 << 20
    k = 8192  # V^T X buffers alone: 30 blocks x rank x k doubles, well above 64 MiB
    Xt = torch.zeros((k, P.n), dtype=torch.float64, device="cuda")
    Yt = torch.full_like(Xt, 7.0)
    with pytest.raises(hq.HQError) as ei:
        P.apply_noalloc(Xt, Yt)
    assert ei.value.status == -1 and "static maximum" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((Yt == 7.0).all())        # nothing ran
    P.close()
