"""Host-side logic of bench.py (no GPU): the one-GPU guard, the workload and
sweep option tables, the reference matching and the stored-inverse count that
the roofline's algorithmic bytes rest on."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2607_27440_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_workload_table_names_existing_generators_and_references():
    for name, (gen, opts) in bench.WORKLOADS.items():
        fn = gen.partition(":")[0]
        assert callable(getattr(W, fn)), name
        assert opts["pc_kernel"] in (0, 1, 2)
        assert opts["m_min"] < opts.get("m_max", 10 ** 9)
    for name, path in bench.REFERENCES.items():
        assert name in bench.WORKLOADS
        assert os.path.exists(os.path.join(ROOT, "tests", "golden", path)), path
    # the M = 4 line: the exact structured inverse and the search space of its sweep
    gen, opts = bench.WORKLOADS["c3"]
    assert gen == "config3" and opts["pc_kernel"] == 2
    ref = bench.reference_eigs("c3")
    assert ref is not None and len(ref) >= W.config3().nev


def test_sweep_options_per_precision():
    fp64, mixed = bench.sweep_opts(0), bench.sweep_opts(1)
    assert fp64 == bench.SWEEP_OPTS
    assert mixed == dict(bench.SWEEP_OPTS, **bench.SWEEP_MIXED)
    assert "inner_max_it" not in mixed       # three refined FP32 cycles (library default)


def test_error_vs_reference_matches_one_to_one_nearest_first():
    ref = np.array([1.0 + 1.0j, 1.0 - 1.0j, 2.0 + 0.0j])
    lam = np.array([1.0 + 1.0j + 1e-9, 1.0 + 1.0j + 2e-9, 2.0 + 0.0j])
    err = bench.error_vs_reference(lam, ref)
    # the second value cannot reuse the first reference: it takes the nearest
    # unused one (2, at distance sqrt 2), and the third the one left (1 - i)
    assert err[0] == pytest.approx(1e-9 / abs(ref[0]), rel=1e-2)
    assert err[1] == pytest.approx(abs(lam[1] - ref[2]) / abs(ref[2]), rel=1e-2)
    assert err[2] == pytest.approx(abs(lam[2] - ref[1]) / abs(ref[1]), rel=1e-2)
    # a complete match of the same set gives zero errors in any order
    assert bench.error_vs_reference(ref[::-1], ref) == [0.0, 0.0, 0.0]


def test_line_slots_pair_mirrored_velocities_for_a_real_target():
    wl = W.config3()
    assert bench._line_slots(wl, 0.05j) == wl.Nxi
    slots = bench._line_slots(wl, 0.0)
    # 61 x 24 trapezoid nodes: xi_y never zero, every node has its mirror
    assert np.all(wl.xi_y != 0.0)
    assert slots == wl.Nxi // 2 == 732
    # a table with a xi_y = 0 row keeps those nodes unpaired
    wl2 = W.config1()
    n_zero = int(np.sum(wl2.xi_y == 0.0))
    assert bench._line_slots(wl2, 0.0) == n_zero + (wl2.Nxi - n_zero) // 2
