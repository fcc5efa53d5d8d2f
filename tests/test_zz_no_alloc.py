"""The allocation-free operator entry point (klst_apply_many_noalloc) against
klst_apply_many, through the C ABI: the same kernels on the same inputs, so the
products must agree bit for bit, on consecutive calls with shrinking inputs,
and sizes beyond the scratch array must be refused."""
import numpy as np
import pytest

from paper_2607_27440_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _pair(ctx, wl, nvec, tau, seed):
    x = _dev(np.concatenate([W.random_vector(wl.n, seed + i) for i in range(nvec)]))
    y_ref = torch.empty_like(x)
    y_na = torch.full_like(x, complex(np.nan, np.nan))
    ctx.apply_many(tau, nvec, x, y_ref)
    ctx.apply_many_noalloc(tau, nvec, x, y_na)
    torch.cuda.synchronize()
    return y_ref, y_na


def test_noalloc_equals_apply_many_on_consecutive_calls():
    from paper_2607_27440_amd import klst
    wl2 = W.config2()
    print(f"[case] noalloc {wl2.name} nvec 16 then 3", flush=True)
    with klst.Context() as ctx:
        ctx.assemble(wl2)
        for nvec, tau, seed in ((16, 0.3 - 0.1j, 100), (3, 0.05j, 200)):
            y_ref, y_na = _pair(ctx, wl2, nvec, tau, seed)
            assert torch.equal(y_ref, y_na), (nvec, float((y_ref - y_na).abs().max()))
    wl1 = W.config1()
    print(f"[case] noalloc {wl1.name} nvec 2 (smaller problem, same scratch)", flush=True)
    with klst.Context() as ctx:
        ctx.assemble(wl1)
        y_ref, y_na = _pair(ctx, wl1, 2, 0.0, 300)
        assert torch.equal(y_ref, y_na)


def test_noalloc_refuses_sizes_beyond_the_scratch():
    from paper_2607_27440_amd import klst
    wl = W.config2()          # Ny = 64, r = 4: 2,304 scratch entries per vector, 227 vectors fit
    print(f"[case] noalloc size limit {wl.name}", flush=True)
    with klst.Context() as ctx:
        ctx.assemble(wl)
        x = torch.zeros(228 * wl.n, dtype=torch.complex128, device=DEV)
        y = torch.empty_like(x)
        with pytest.raises(klst.KlstError) as ei:
            ctx.apply_many_noalloc(0.0, 228, x, y)
        assert ei.value.status == klst.EINVAL
        ctx.apply_many_noalloc(0.0, 227, x, y)
        torch.cuda.synchronize()
        assert torch.count_nonzero(y).item() == 0
