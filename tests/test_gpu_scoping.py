"""The paper's scoping workload (Section 4): 3-D Franke function, separate
random query grid, float64 path and storage.  GPU fit and evaluation against
the oracle, and the convergence the experiments show (errors fall and the
tree grows as tau falls)."""
import numpy as np
import pytest

import oracle
import synthetic
from test_gpu_parity import FP64_RMS, compare_eval, compare_topology, dev, fitted_rms, oracle_fit, print_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fmt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1511_01353_amd as m
    m.load_library()
    return m


@pytest.mark.parametrize("n,p", [(8 ** 4, 4), (8 ** 4, 8), (8 ** 5, 4)])
def test_scoping_matches_oracle_and_converges(fmt, n, p):
    errs, nodes = [], []
    for tau in (1e-6, 1e-10):
        pr = synthetic.scoping_problem(n, p, tau, 6100 + p, depth=10)
        print_case("scoping", pr)
        o = fmt.fmt_default_opts(p=p, tol=tau, max_depth=10)
        tr = fmt.fmt_fit(o, dev(pr.x), dev(pr.y), dev(pr.z), dev(pr.f))
        ot = oracle_fit(pr)
        gn, pts = compare_topology(tr, ot)
        assert fitted_rms(pr, pts, ot) <= FP64_RMS
        got = tr.eval(dev(pr.qx), dev(pr.qy), dev(pr.qz)).cpu().numpy()
        compare_eval(ot, gn, pr, got, oracle.evaluate(ot, pr.qx, pr.qy, pr.qz), FP64_RMS, min_frac=0.95)
        err = got - pr.qf_true
        errs.append(float(np.sqrt(np.mean(err * err))))
        nodes.append(int(tr.info().nodes))
        print(f"tau {tau:g}: nodes {nodes[-1]}, E_rms {errs[-1]:.3e}, E_inf {np.max(np.abs(err)):.3e}", flush=True)
        tr.close()
    assert nodes[1] >= nodes[0]
    assert errs[1] <= errs[0]
