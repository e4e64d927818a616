"""Host-side logic that needs no GPU: the benchmark's lookup of measured HBM
traffic, the binding's checks of device tensors, and the workload generators
of the paper's scaling and level-set experiments."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import bench
from gen.configs import config5, config_grid, config_tychastic


def test_counter_traffic_matches_only_the_profiled_run(tmp_path, monkeypatch):
    src = tmp_path / "kernel.h"
    src.write_text("// kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    recs = [dict(kernel="k_pdhg_wide", variant="cont", check_every=75, c_tau=2.0, hbm_bytes_per_launch=10,
                 kernel_source_sha256=sha),
            dict(kernel="k_pdhg_wide", variant="mlp", check_every=75, c_tau=2.0, hbm_bytes_per_launch=20,
                 kernel_source_sha256="0" * 64)]
    prof = tmp_path / "prof.md"
    prof.write_text("# summary\n\n" + "".join("traffic:" + json.dumps(r) + "\n" for r in recs))
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    monkeypatch.setattr(bench, "COUNTERS", str(prof))
    assert bench.counter_traffic("cont", 75, 2.0, "k_pdhg_wide")["hbm_bytes_per_launch"] == 10
    assert bench.counter_traffic("cont", 75, 2.0, "k_pdhg") is None          # other kernel
    assert bench.counter_traffic("cont", 50, 2.0, "k_pdhg_wide") is None     # other launch length
    assert bench.counter_traffic("cont", 75, 5.0, "k_pdhg_wide") is None     # other step ratio
    assert bench.counter_traffic("mlp", 75, 2.0, "k_pdhg_wide") is None      # kernel changed since
    assert bench.counter_traffic("cold", 75, 2.0, "k_pdhg_wide") is None     # not profiled
    src.write_text("// edited kernel\n")
    assert bench.counter_traffic("cont", 75, 2.0, "k_pdhg_wide") is None


def test_committed_traffic_records_are_for_the_headline_settings():
    w = config5(npts=16)
    with open(bench.COUNTERS) as f:
        recs = [json.loads(l[len("traffic:"):]) for l in f if l.startswith("traffic:")]
    assert recs
    for r in recs:
        assert r["check_every"] == w.opts["check_every"] and r["c_tau"] == w.opts["c_tau"]
        # each figure is rounded to whole bytes on its own
        assert abs(r["hbm_bytes_per_launch"] - r["read_bytes_per_launch"] - r["write_bytes_per_launch"]) <= 1


def test_device_tensor_checks_refuse_host_or_mistyped_tensors():
    torch = pytest.importorskip("torch")
    from paper_1712_08226_amd.hopfpd import Solver
    s = Solver.__new__(Solver)          # the checks need no context
    assert s._dev_ptr(None, "lam", "torch.float64", 4, 3) is None
    with pytest.raises(ValueError):
        s._dev_ptr(torch.zeros(4, 3, dtype=torch.float64), "x", "torch.float64", 4, 3)   # host tensor


def test_tychastic_generator_structure():
    k = 15
    w = config_tychastic(2 * k, npts=8)
    S = w.systems[0]
    A2 = np.array([[0.0, 1.0], [0.0, 0.0]])
    np.testing.assert_array_equal(S.A, np.kron(np.eye(k), A2))
    np.testing.assert_array_equal(S.B, np.kron(np.ones((k, 1)), np.array([[0.0], [1.0]])))
    np.testing.assert_allclose(S.W, 0.04 * k * np.eye(2 * k))
    assert (S.uset, S.quad, S.N, S.t_max) == ("box", "left", 100, 2.0)
    chi = w.x.reshape(8, k, 2)
    assert w.x.shape == (8, 2 * k) and abs(chi[..., 0].mean() - 1.0) < 0.1 and abs(chi[..., 1].mean()) < 0.1
    with pytest.raises(ValueError):
        config_tychastic(31)


def test_grid_generator():
    w = config_grid(5)
    assert w.x.shape == (25, 2)
    np.testing.assert_allclose(w.x.min(axis=0), [-1, -1])
    np.testing.assert_allclose(w.x.max(axis=0), [1, 1])
    S = w.systems[0]
    np.testing.assert_allclose(S.W, 0.04 * np.eye(2))
    assert S.quad == "left" and S.N == 100


def test_tuner_accepts_only_the_reference_results():
    """A tuning candidate is eligible only with the reference setting's
    statuses, T within the search tolerance and gaps within the tolerance
    (min time), or overlapping certified intervals (value)."""
    from paper_1712_08226_amd.tune import _same
    ref = dict(status=np.array([0, 0, 2]), T=np.array([1.0, 2.0, np.inf]), gap=np.array([1e-7, 1e-7, np.nan]))
    assert _same(ref, dict(ref, T=np.array([1.00005, 2.0, np.inf])), "min_time")
    assert not _same(ref, dict(ref, T=np.array([1.001, 2.0, np.inf])), "min_time")
    assert not _same(ref, dict(ref, status=np.array([0, 3, 2])), "min_time")
    assert not _same(ref, dict(ref, gap=np.array([2e-6, 1e-7, np.nan])), "min_time")
    v = dict(status=np.array([0, 0]), phi_lo=np.array([1.0, -2.0]), phi_hi=np.array([1.1, -1.9]))
    assert _same(v, dict(v, phi_lo=np.array([1.05, -1.95]), phi_hi=np.array([1.2, -1.8])), "value")
    assert not _same(v, dict(v, phi_lo=np.array([1.2, -2.0]), phi_hi=np.array([1.3, -1.9])), "value")


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; asking for more exits with status 2 and
    says why, before touching a device."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_unscented_config_and_weights():
    """The unscented workload: five sigma points per query around means in
    the stated box, target blocks ell / w_i with the 1/3, 1/6 weights."""
    from gen.configs import config_unscented
    w = config_unscented(npts=16)
    spec = w.systems[0]
    assert w.x.shape == (16, 10) and spec.A.shape == (10, 10) and spec.B.shape == (10, 1)
    assert np.allclose(np.diag(spec.W), 0.04 / np.repeat([1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6], 2))
    mu = w.x[:, :2]
    assert np.all((mu[:, 0] >= 0.8) & (mu[:, 0] <= 1.2) & (mu[:, 1] >= -0.2) & (mu[:, 1] <= 0.2))
