"""The minimum-time entry point that allocates nothing
(hopf_min_time_dev_noalloc, solver state in the library's fixed device
scratch) against hopf_min_time_dev on the same points: identical statuses,
|dT| <= 1e-4 T and final gaps <= 1e-6, on two calls in a row (the second
with fewer points, so it runs on what the first left in the scratch), and a
call too large for the scratch is refused."""
import sys

import numpy as np
import pytest

from gen.configs import config5
from gen.workloads import planted_drift_points

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_no_alloc_matches_min_time_dev():
    import torch
    from paper_1712_08226_amd import Solver
    from paper_1712_08226_amd.hopfpd import HopfError
    say("case: no-allocation entry point vs hopf_min_time_dev")
    spec = config5(npts=8).systems[0]
    x_all, _ = planted_drift_points(spec, 1200, 0.2, 3.0, 31)
    s = Solver(0)
    try:
        s.set_systems([spec])
        s.set_opts(prec="fp32", c_tau=2.0, check_every=75, warm="cont")
        dev = torch.device("cuda:0")
        stream = torch.cuda.current_stream(dev)
        for k, npts in enumerate((1200, 300)):
            x = torch.tensor(x_all[:npts], dtype=torch.float64, device=dev)
            out = {}
            for name in ("dev", "noalloc"):
                T = torch.empty(npts, dtype=torch.float64, device=dev)
                gap = torch.empty_like(T)
                st = torch.empty(npts, dtype=torch.int32, device=dev)
                lam = torch.empty(npts, spec.n, dtype=torch.float64, device=dev)
                if name == "dev":
                    s.min_time_dev(x, T, gap, st, lam=lam, stream=stream)
                else:
                    s.min_time_dev_noalloc(x, T, gap, st, lam=lam, stream=stream)
                out[name] = dict(T=T.cpu().numpy(), gap=gap.cpu().numpy(), status=st.cpu().numpy(),
                                 lam=lam.cpu().numpy())
            a, b = out["dev"], out["noalloc"]
            say("call", k, "points", npts, "statuses", np.bincount(b["status"], minlength=5))
            assert np.array_equal(a["status"], b["status"])
            ok = a["status"] == 0
            assert ok.all()
            assert np.all(np.abs(a["T"][ok] - b["T"][ok]) <= 1e-4 * a["T"][ok])
            assert np.all(b["gap"][ok] <= 1e-6)
        big = torch.zeros(20000, spec.n, dtype=torch.float64, device=dev)
        T = torch.empty(20000, dtype=torch.float64, device=dev)
        with pytest.raises(HopfError, match="scratch"):
            s.min_time_dev_noalloc(big, T, torch.empty_like(T), torch.empty(20000, dtype=torch.int32, device=dev))
    finally:
        s.close()
