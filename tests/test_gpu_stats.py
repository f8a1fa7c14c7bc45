"""Run statistics: the method's bytes per iteration follow their definition (per touched factor
edge 4 + 3s, per written edge s or 2s, s per NOISY_OR activation), checked against counts made here
from the schedule's levels; message updates equal non-PRIOR edges times iterations."""
import numpy as np
import pytest

import paper_2509_22337_amd as F
from paper_2509_22337_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.load()


def _expected(w, levels, s, needs_old):
    deg = np.diff(w.fac_off)
    edge_fac = np.repeat(np.arange(w.num_factors), deg)
    nonprior = w.fac_type[edge_fac] != W.PRIOR
    touched = noisy = 0
    for a in range(w.num_factors):
        if w.fac_type[a] == W.PRIOR:
            continue
        lv = np.unique(levels[w.fac_off[a]:w.fac_off[a + 1]])
        touched += len(lv) * deg[a]
        if w.fac_type[a] == W.NOISY_OR:
            noisy += len(lv) * (deg[a] - 1)
    written = int(nonprior.sum())
    return touched * (4 + 3 * s) + written * (2 * s if needs_old else s) + noisy * s, written


@pytest.mark.parametrize("precision,s", [("fp64", 8), ("fp32", 4)])
def test_method_bytes_per_iter(precision, s):
    for w, tol, damping in ((W.datalog(2, num_tuples=400, num_rules=300), 0.0, 0.0),
                            (W.datalog(2, num_tuples=400, num_rules=300), 0.0, 0.5),
                            (W.smartfl(3, levels=20, width=40, max_iters=10), 1e-6, 0.0)):
        g = F.Graph.from_workload(w, precision=precision)
        st = g.run(5, tol, damping)
        levels = g.schedule_levels()
        g.close()
        exp, written = _expected(w, levels, s, tol > 0 or damping > 0)
        assert st["method_bytes_per_iter"] == pytest.approx(exp, rel=1e-12)
        assert st["message_updates"] == written * st["iterations"]
        if w.edge_rank is None:  # flooding: 4 + 5s per edge, + s per activation
            nonprior = int(np.diff(w.fac_off)[w.fac_type != W.PRIOR].sum())
            ep = int(np.diff(w.fac_off)[w.fac_type == W.NOISY_OR].sum() - (w.fac_type == W.NOISY_OR).sum())
            old = 2 if (tol > 0 or damping > 0) else 1
            assert exp == nonprior * (4 + 3 * s + old * s) + ep * s
