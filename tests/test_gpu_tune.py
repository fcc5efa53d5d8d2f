"""The launch autotuner (klst_autotune) on the GPU: it reports a valid choice no
slower than the heuristic beyond timing noise; tile choices leave the operator
bit-identical; and under a tuned table (moment splits and GEMV waves changed)
the served sweep is still bit-identical alone and in a concurrent mix."""
import numpy as np
import pytest

from paper_2607_27440_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture
def klst():
    from paper_2607_27440_amd import klst as K
    K.tune_clear()
    yield K
    K.tune_clear()


def test_autotune_entry_is_valid(klst):
    wl = W.config2()
    print(f"[case] autotune {wl.name}", flush=True)
    with klst.Context(pc_kernel=2) as ctx:
        ctx.assemble(wl)
        ctx.precond_setup(wl.sigma)
        e = ctx.autotune(nvec=1, reps=10)
        print(e, flush=True)
        assert (e["Ny"], e["Nxi"], e["nvec"], e["precision"]) == (wl.Ny, wl.Nxi, 1, 0)
        assert e["apply_tile"] in (1, 2, 3, 6) and e["apply_waves"] in (1, 4)
        assert 1 <= e["moment_splits"] <= 8 and e["gemv_waves"] in (4, 8, 16)
        assert e["us_tuned"] <= 1.25 * e["us_default"]


def test_tile_choices_leave_the_operator_bit_identical(klst):
    wl = W.config2()
    nvec = 6
    x = torch.from_numpy(np.concatenate([W.random_vector(wl.n, 70 + i) for i in range(nvec)])).to(DEV)
    with klst.Context() as ctx:
        ctx.assemble(wl)
        y_ref = torch.empty_like(x)
        ctx.apply_many(0.1j, nvec, x, y_ref)
        torch.cuda.synchronize()
        ctx.autotune(nvec=nvec, reps=5)
        y = torch.empty_like(x)
        ctx.apply_many(0.1j, nvec, x, y)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref)
        # single applies (their own tuned entry, same moment splits) equal the batch
        y1 = torch.empty(wl.n, dtype=torch.complex128, device=DEV)
        for i in range(nvec):
            ctx.apply(0.1j, x[i * wl.n:(i + 1) * wl.n], y1)
            torch.cuda.synchronize()
            assert torch.equal(y1, y_ref[i * wl.n:(i + 1) * wl.n])


@pytest.mark.parametrize("tile", [None, (1, 1), (2, 4), (3, 1), (6, 4), (0, 8)])
def test_every_operator_kernel_gives_the_same_bits(klst, tmp_path, tile):
    """At the M = 4 shape (Ny = 96, 6 row tiles, 5 moment parts), the many-vector
    operator under each launch choice (the streaming kernel by default or as
    (0, 8); the tiled MFMA kernel with 1-6 row tiles and 1 or 4 wavefronts)
    gives every vector bit for bit what a single application gives it."""
    wl = W.config3()
    nvec = 9
    print(f"[case] operator kernel choice {tile} at {wl.name}", flush=True)
    x = torch.from_numpy(np.concatenate([W.random_vector(wl.n, 90 + i) for i in range(nvec)])).to(DEV)
    with klst.Context() as ctx:
        ctx.assemble(wl)
        y1 = torch.empty_like(x)
        for i in range(nvec):
            ctx.apply(0.3 + 0.1j, x[i * wl.n:(i + 1) * wl.n], y1[i * wl.n:(i + 1) * wl.n])
        if tile is not None:
            path = tmp_path / "tile.txt"
            path.write_text(f"# one entry\n{wl.Ny} {wl.Nxi} {nvec} 0 {tile[0]} {tile[1]} 0 0\n")
            klst.tune_load(str(path))
        y = torch.empty_like(x)
        ctx.apply_many(0.3 + 0.1j, nvec, x, y)
        torch.cuda.synchronize()
        assert torch.equal(y, y1)


def test_sweep_bit_identical_alone_and_in_mix_under_a_tuned_table(klst, tmp_path):
    wls = sorted(W.sweep(seed=4, count=64, nev=6), key=lambda w: w.n)[:6]
    opts = dict(m_max=30, pc_kernel=2, max_it=1500)
    # tune every shape of the set, then fix the table (saved and reloaded)
    for wl in wls:
        with klst.Context(**opts) as ctx:
            ctx.assemble(wl)
            ctx.precond_setup(wl.sigma)
            ctx.autotune(nvec=1, reps=5)
    path = tmp_path / "tune.txt"
    klst.tune_save(str(path))
    klst.tune_clear()
    klst.tune_load(str(path))
    print("[case] tuned sweep sizes", [w.n for w in wls], flush=True)
    with klst.Server(slots=1, **opts) as alone:
        ref = [alone.solve_all([wl])[0] for wl in wls]
    with klst.Server(slots=4, **opts) as mix:
        got = mix.solve_all(wls)
    for r, g in zip(ref, got):
        assert r["nconv"] == g["nconv"] and np.array_equal(r["lam"], g["lam"])
        assert np.array_equal(r["resid"], g["resid"])
