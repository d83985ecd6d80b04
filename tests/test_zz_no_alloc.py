"""pr_prox_noalloc (the prox entry point that allocates nothing) against
pr_prox through the C ABI: bit-identical outputs on two calls in a row, the
second with a smaller input, plus its error paths."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(p, seed, n0, n1):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(p) * rng.choice([0.1, 1.0, 3.0], size=p)
    st = np.zeros(p, dtype=np.int8)
    perm = rng.permutation(p)
    st[perm[:n0]] = 1
    st[perm[n0:n0 + n1]] = 2
    return v, st


def _raw(fn, v, p, rho, k, M, st, out):
    import paper_2603_01306_amd as pr
    import torch
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return getattr(pr.load(), fn)(s, ctypes.c_void_p(v.data_ptr()), int(p), float(rho), int(k), float(M),
                                  ctypes.c_void_p(st.data_ptr()), ctypes.c_void_p(out.data_ptr()))


@pytest.mark.parametrize("M", [2.0, float("inf")])
def test_noalloc_prox_equals_pr_prox_two_calls(dev, M):
    import torch
    print(f"noalloc prox: M={M}", flush=True)
    sizes = [(20011, 5, 40, 3, 0.7), (1537, 9, 11, 2, 4.0)]  # second call smaller
    for p, seed, n0, n1, rho in sizes:
        v, st = _case(p, seed, n0, n1)
        k = 10
        vd = torch.from_numpy(v).to(dev)
        sd = torch.from_numpy(st).to(dev)
        ref = torch.empty_like(vd)
        got = torch.full_like(vd, float("nan"))
        assert _raw("pr_prox", vd, p, rho, k, M, sd, ref) == 0
        assert _raw("pr_prox_noalloc", vd, p, rho, k, M, sd, got) == 0
        torch.cuda.synchronize()
        r = ref.cpu().numpy()
        g = got.cpu().numpy()
        assert np.array_equal(r, g), (p, np.max(np.abs(r - g)))
        # kbar > 0 and both J0 and J1 present: the case is not degenerate
        assert np.count_nonzero(g[st == 0]) >= 1 and np.all(g[st == 1] == 0.0)


def test_noalloc_prox_errors(dev):
    import paper_2603_01306_amd as pr
    import torch
    p = 64
    v, st = _case(p, 1, 3, 0)
    vd = torch.from_numpy(v).to(dev)
    out = torch.full_like(vd, 7.0)
    # |J1| > k: rejected on the device, out left alone
    st_bad = st.copy()
    st_bad[:5] = 2
    sd = torch.from_numpy(st_bad).to(dev)
    rc = _raw("pr_prox_noalloc", vd, p, 0.5, 4, 2.0, sd, out)
    assert rc == -1
    assert torch.all(out == 7.0)
    # a status code outside {0, 1, 2}
    st_bad = st.copy()
    st_bad[7] = 5
    rc = _raw("pr_prox_noalloc", vd, p, 0.5, 4, 2.0, torch.from_numpy(st_bad).to(dev), out)
    assert rc == -1
    assert torch.all(out == 7.0)
    # p beyond the workspace: rejected on the host before any launch
    rc = _raw("pr_prox_noalloc", vd, pr.PROX_NOALLOC_MAX_P + 1, 0.5, 4, 2.0, sd, out)
    assert rc == -1
    # a valid call after the failures still matches pr_prox
    sd = torch.from_numpy(st).to(dev)
    ref = torch.empty_like(vd)
    assert _raw("pr_prox", vd, p, 0.5, 4, 2.0, sd, ref) == 0
    assert _raw("pr_prox_noalloc", vd, p, 0.5, 4, 2.0, sd, out) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
