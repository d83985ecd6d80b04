"""Iteration variants of the convergence study on the GPU (pr_opts.method):
FISTA with the duality-gap restart, FISTA without restart, FISTA with
function-value restart, proximal gradient.  Per-iterate (Phi, Psi) traces
against the FP64 oracle running the same variant, and the certified bound of
every variant against the oracle's."""
import math

import numpy as np
import pytest

import oracle
from workloads import config_instance, make_instance

pytestmark = pytest.mark.gpu

METHODS = [("gap", 0, oracle.FISTA_GAP), ("fista", 1, oracle.FISTA), ("fv", 2, oracle.FISTA_FV), ("pgd", 3, oracle.PGD)]


@pytest.fixture(scope="module")
def c1(dev):
    import torch
    import paper_2603_01306_amd as pr
    inst = config_instance("ls_root_n500_p200_f64")
    ctx = pr.Context(torch.from_numpy(inst.Xcm).to(dev), torch.from_numpy(inst.y).to(dev), 0)
    L = 2.02 * float(np.linalg.eigvalsh(inst.X64() @ inst.X64().T).max())
    yield inst, ctx, L
    ctx.close()


@pytest.mark.parametrize("name,gm,om", METHODS)
def test_trace_matches_oracle(c1, name, gm, om):
    import torch
    import paper_2603_01306_amd as pr
    inst, ctx, L = c1
    its = 60
    tr = torch.full((2 * (its + 1),), float("nan"), dtype=torch.float64, device="cuda")
    node = pr.Node(10, 1.0, 2.0, J0=[3, 7], J1=[20])
    r = ctx.solve(node, rel_gap_tol=0.0, max_iter=its, L=L, method=gm, trace=tr)
    ref = oracle.solve(inst.Xcm, inst.y, 0, 1.0, 2.0, 10, status=node.status(inst.p), L=L, tol=0.0,
                       max_iter=its, trace_cap=its + 1, method=om)
    assert r["iters"] == ref["iters"] == its
    assert r["restarts"] == ref["restarts"]
    t = tr.cpu().numpy().reshape(-1, 2)
    phi, psi = t[:, 0], t[:, 1]
    ophi = ref["phi_trace"]
    opsi = ophi - ref["trace"]
    fin = np.isfinite(ophi)
    assert np.array_equal(np.isfinite(phi), fin)
    assert np.all(np.abs(phi[fin] - ophi[fin]) <= 1e-10 * np.abs(ophi[fin]))
    assert np.all(np.abs(psi - opsi) <= 1e-10 * np.abs(ophi[-1]))


@pytest.mark.parametrize("name,gm,om", METHODS)
def test_every_variant_reaches_the_oracle_bound(c1, name, gm, om):
    import paper_2603_01306_amd as pr
    inst, ctx, L = c1
    node = pr.Node(10, 1.0, 2.0)
    r = ctx.solve(node, rel_gap_tol=1e-7, max_iter=60000, L=L, method=gm)
    ref = oracle.solve(inst.Xcm, inst.y, 0, 1.0, 2.0, 10, L=L, tol=1e-10)
    assert r["status"] == pr.CONVERGED, r
    assert abs(r["lower_bound"] - ref["lb"]) <= 1e-7 * abs(ref["ub"])
    assert r["lower_bound"] <= ref["ub"] * (1 + 1e-12)


def test_logistic_function_value_restart_trace(dev):
    import torch
    import paper_2603_01306_amd as pr
    inst = make_instance(n=400, p=120, corr=0.5, k_true=5, snr=5.0, loss=1, seed=8, storage="f64")
    ctx = pr.Context(torch.from_numpy(inst.Xcm).to(dev), torch.from_numpy(inst.y).to(dev), 1)
    L = 1.01 * 0.25 * float(np.linalg.eigvalsh(inst.X64() @ inst.X64().T).max())
    its = 50
    tr = torch.full((2 * (its + 1),), float("nan"), dtype=torch.float64, device="cuda")
    node = pr.Node(5, 0.3, 2.0, J1=[0])
    r = ctx.solve(node, rel_gap_tol=0.0, max_iter=its, L=L, method=pr.FISTA_FV, trace=tr)
    ref = oracle.solve(inst.Xcm, inst.y, 1, 0.3, 2.0, 5, status=node.status(inst.p), L=L, tol=0.0,
                       max_iter=its, trace_cap=its + 1, method=oracle.FISTA_FV)
    t = tr.cpu().numpy().reshape(-1, 2)
    fin = np.isfinite(ref["phi_trace"])
    assert np.all(np.abs(t[fin, 0] - ref["phi_trace"][fin]) <= 1e-10 * np.abs(ref["phi_trace"][fin]))
    assert r["restarts"] == ref["restarts"]
    ctx.close()


def test_rejects_unknown_method(c1):
    import paper_2603_01306_amd as pr
    inst, ctx, L = c1
    with pytest.raises(pr.PrError):
        ctx.solve(pr.Node(10, 1.0, 2.0), method=8)
