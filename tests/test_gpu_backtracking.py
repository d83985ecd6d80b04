"""FISTA with backtracking (pr_opts.method PR_FISTA_BT_GAP / PR_FISTA_BT) on
the GPU against the oracle's FISTA with backtracking: per accepted iterate
(Phi, Psi), the accepted / rejected / restart counts and the final step
constant, for both losses, FP64 and FP32 designs and the Gram mode; at full
size the certificates recomputed by the oracle over the stored X."""
import math

import numpy as np
import pytest

import oracle
from workloads import config_instance, make_instance

pytestmark = pytest.mark.gpu


def _ctx(dev, inst, gram=False):
    import torch
    import paper_2603_01306_amd as pr
    c = pr.Context(torch.from_numpy(inst.Xcm).to(dev), torch.from_numpy(inst.y).to(dev), inst.loss)
    if gram:
        c.enable_gram()
    return c


def _zeta(inst, beta):
    u = inst.X64().T @ beta
    return 2.0 * (inst.y - u) if inst.loss == 0 else inst.y / (1.0 + np.exp(inst.y * u))


@pytest.mark.parametrize("loss,storage,restart,gram", [(0, "f64", True, False), (0, "f32", False, False),
                                                       (1, "f64", True, False), (1, "f32", False, False),
                                                       (1, "f32", True, False), (0, "f32", True, True)])
def test_backtracking_trace_matches_oracle(dev, loss, storage, restart, gram):
    import torch
    import paper_2603_01306_amd as pr
    inst = make_instance(n=512, p=256, corr=0.7, k_true=6, snr=5.0, loss=loss, seed=70 + loss, storage=storage)
    ctx = _ctx(dev, inst, gram)
    node = pr.Node(6, 0.4, 2.0, J0=[3, 17, 40], J1=[8])
    st = node.status(inst.p)
    Lmax = (2.0 if loss == 0 else 0.25) * float(np.linalg.eigvalsh(inst.X64() @ inst.X64().T).max()) * 1.01
    L0, its = Lmax / 32.0, 120
    tr = torch.full((2 * (its + 1),), float("nan"), dtype=torch.float64, device=dev)
    method = pr.FISTA_BT_GAP if restart else pr.FISTA_BT
    r = ctx.solve(node, rel_gap_tol=0.0, max_iter=its, L=Lmax, L0=L0, acfgm_c=2.0, method=method, trace=tr)
    ref = oracle.solve_bt(inst.Xcm, inst.y, loss, 0.4, 2.0, 6, status=st, L0=L0, c=2.0, Lmax=Lmax,
                          restart=restart, tol=0.0, max_iter=its, trace_cap=its + 1)
    print({k: v for k, v in r.items() if k not in ("beta", "zeta")}, ref["iters"], ref["restarts"], ref["rejected"],
          ref["L"], flush=True)
    assert r["iters"] == ref["iters"] == its
    assert r["restarts"] == ref["restarts"] and r["trials"] == ref["rejected"] and r["trials"] >= 1
    assert r["L"] == pytest.approx(ref["L"], rel=1e-15)
    t = tr.cpu().numpy().reshape(-1, 2)
    ophi = ref["phi_trace"]
    opsi = ophi - ref["trace"]
    fin = np.isfinite(ophi)
    assert np.array_equal(np.isfinite(t[:, 0]), fin)
    tol = 1e-9 if gram else 1e-10
    assert np.all(np.abs(t[fin, 0] - ophi[fin]) <= tol * np.abs(ophi[fin]))
    assert np.all(np.abs(t[:, 1] - opsi) <= tol * np.abs(ophi[-1]))
    ctx.close()


@pytest.mark.parametrize("loss", [0, 1])
def test_backtracking_converges_to_the_oracle_bound(dev, loss):
    """To a 1e-8 gap with the library's own step cap: the bound is the
    oracle's, and the returned (beta, zeta) certify it over the stored X."""
    import paper_2603_01306_amd as pr
    inst = make_instance(n=600, p=256, corr=0.6, k_true=6, snr=5.0, loss=loss, seed=80 + loss, storage="f64")
    ctx = _ctx(dev, inst)
    node = pr.Node(6, 0.5, 2.0, J0=[1, 2], J1=[5])
    st = node.status(inst.p)
    r = ctx.solve(node, rel_gap_tol=1e-8, want_zeta=True, method=pr.FISTA_BT_GAP)
    ref = oracle.solve(inst.Xcm, inst.y, loss, 0.5, 2.0, 6, status=st, tol=1e-11)
    assert r["status"] == pr.CONVERGED and r["rel_gap"] <= 1e-8
    assert abs(r["lower_bound"] - ref["lb"]) <= 1e-8 * abs(ref["ub"])
    psi = oracle.dual(inst.Xcm, inst.y, r["zeta"].cpu().numpy(), loss, 0.5, 2.0, 6, status=st)
    phi = oracle.primal(inst.Xcm, inst.y, r["beta"].cpu().numpy(), loss, 0.5, 2.0, 6, status=st)
    assert abs(psi - r["lower_bound"]) <= 1e-11 * abs(phi) and abs(phi - r["primal"]) <= 1e-11 * abs(phi)
    ctx.close()


@pytest.mark.parametrize("name", ["ls_root_n16384_p8192_f32", "logistic_root_n32768_p16384_f32"])
def test_backtracking_full_size_certificate(dev, name):
    """The two full-size roots to 1e-6 with FISTA with backtracking and the gap
    restart: the oracle recomputes Psi at the returned dual vector and Phi at
    the returned beta; fewer iterations than the fixed step."""
    import paper_2603_01306_amd as pr
    inst = config_instance(name)
    ctx = _ctx(dev, inst)
    k = 20 if inst.loss == 0 else 15
    node = pr.Node(k, 0.1, 2.0)
    r = ctx.solve(node, want_zeta=True, method=pr.FISTA_BT_GAP)
    f = ctx.solve(node, want_beta=False)
    print(name, {q: v for q, v in r.items() if q not in ("beta", "zeta")}, "fixed-step iters", f["iters"], flush=True)
    assert r["status"] == pr.CONVERGED and f["status"] == pr.CONVERGED
    psi = oracle.dual(inst.Xcm, inst.y, r["zeta"].cpu().numpy(), inst.loss, 0.1, 2.0, k)
    phi = oracle.primal(inst.Xcm, inst.y, r["beta"].cpu().numpy(), inst.loss, 0.1, 2.0, k)
    assert abs(psi - r["lower_bound"]) <= 1e-10 * abs(psi) and abs(phi - r["primal"]) <= 1e-10 * abs(phi)
    assert 0.0 <= (phi - psi) / abs(phi) <= 1e-6
    assert abs(r["lower_bound"] - f["lower_bound"]) <= 2e-6 * abs(phi)
    assert r["iters"] + r["trials"] < f["iters"]
    ctx.close()


def test_backtracking_rejects_bad_arguments(dev):
    import paper_2603_01306_amd as pr
    inst = make_instance(n=64, p=32, corr=0.5, k_true=3, snr=5.0, loss=0, seed=2, storage="f64")
    c = _ctx(dev, inst)
    for kw in (dict(acfgm_c=1.0), dict(L0=-1.0), dict(acfgm_c=float("inf"))):
        with pytest.raises(pr.PrError):
            c.solve(pr.Node(3, 0.5, 2.0), method=pr.FISTA_BT_GAP, **kw)
    c.close()
