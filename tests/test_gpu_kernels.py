"""GPU parity of the building blocks against the FP64 oracle, through the C ABI:
prox of g_N (Algorithm 2 + Moreau), g_N (Algorithm 1), g_N* (closed-form
conjugate), and the FP64-accumulated X beta / X^T r products."""
import math

import numpy as np
import pytest

import oracle
from workloads import make_instance, round_bf16, bf16_to_f32

pytestmark = pytest.mark.gpu


def _pr():
    import paper_2603_01306_amd as pr
    return pr


def _rand_node(rng, p, k):
    st = np.zeros(p, np.int8)
    idx = rng.permutation(p)
    n0 = int(rng.integers(0, p // 2 + 1))
    n1 = int(rng.integers(0, min(k, p - n0) + 1))
    st[idx[:n0]] = oracle.ZERO
    st[idx[n0:n0 + n1]] = oracle.ONE
    return st


def _prox_case(i):
    rng = np.random.default_rng(1000 + i)
    sizes = [1, 2, 7, 63, 64, 65, 1000, 1023, 1024, 1025, 3000, 8192, 16384, 20011]
    p = sizes[i % len(sizes)]
    k = int(rng.integers(1, max(2, min(p, 40))))
    M = [0.5, 1.0, 2.0, math.inf][i % 4]
    rho = 10.0 ** rng.uniform(-7, 2)
    scale = 10.0 ** rng.uniform(-3, 3)
    v = rng.standard_normal(p) * scale
    if i % 5 == 0:
        v[rng.integers(0, p, size=p // 3)] = 0.0
    if i % 6 == 0:
        v = np.round(v / scale, 1) * scale   # many exact ties
    st = _rand_node(rng, p, k) if i % 3 == 1 else np.zeros(p, np.int8)
    return v, rho, k, M, st


@pytest.mark.parametrize("i", range(56))
def test_prox_matches_algorithm2(dev, i):
    import torch
    pr = _pr()
    v, rho, k, M, st = _prox_case(i)
    assert np.sum(st == oracle.ONE) <= k   # the generator draws |J1| <= k
    x_gpu = pr.prox(torch.from_numpy(v).to(dev), rho, k, M, torch.from_numpy(st).to(dev)).cpu().numpy()
    x_orc = oracle.prox_g(v, rho, k, M, st)
    # element by element, against the largest entry of the result
    xmax = float(np.max(np.abs(x_orc)))
    err = np.abs(x_gpu - x_orc)
    print(f"case {i}: p={v.size} k={k} M={M} rho={rho:.3g} max err={err.max():.2e} "
          f"err/max(1,|x|)={err.max() / max(1.0, xmax):.2e}")
    assert np.all(err <= 1e-12 * max(1.0, xmax))
    # structural facts of Algorithm 2: J0 -> 0 exactly, J1 -> ridge/box map
    assert np.all(x_gpu[st == oracle.ZERO] == 0.0)
    j1 = st == oracle.ONE
    np.testing.assert_allclose(x_gpu[j1], np.sign(v[j1]) * np.minimum(np.abs(v[j1]) / (1 + rho), M),
                               rtol=1e-14, atol=0)


@pytest.mark.parametrize("i", range(0, 56, 5))
def test_prox_fenchel_young_on_gpu_output(dev, i):
    """x = prox_{rho g}(v), a = (v - x)/rho satisfies g(x) + g*(a) = a^T x."""
    import torch
    pr = _pr()
    v, rho, k, M, st = _prox_case(i)
    assert np.sum(st == oracle.ONE) <= k   # the generator draws |J1| <= k
    x = pr.prox(torch.from_numpy(v).to(dev), rho, k, M, torch.from_numpy(st).to(dev)).cpu().numpy()
    a = (v - x) / rho
    a[st == oracle.ZERO] = 0.0
    lhs = oracle.g(x, k, st) + oracle.gstar(a, k, M, st)
    rhs = float(a @ x)
    assert abs(lhs - rhs) <= 1e-9 * max(1.0, abs(lhs), float(np.abs(a) @ np.abs(x)))


def test_prox_edge_cases(dev):
    import torch
    pr = _pr()
    # all zero input
    v = np.zeros(100)
    st = np.zeros(100, np.int8)
    out = pr.prox(torch.from_numpy(v).to(dev), 0.3, 5, 2.0, torch.from_numpy(st).to(dev)).cpu().numpy()
    assert np.all(out == 0)
    # kbar = 0: |J1| = k forces the free part to zero
    rng = np.random.default_rng(5)
    v = rng.standard_normal(50)
    st = np.zeros(50, np.int8)
    st[[1, 2, 3]] = oracle.ONE
    out = pr.prox(torch.from_numpy(v).to(dev), 0.3, 3, 2.0, torch.from_numpy(st).to(dev)).cpu().numpy()
    assert np.all(out[st == 0] == 0)
    # kbar >= pbar: ridge with box on every free coordinate
    out = pr.prox(torch.from_numpy(v).to(dev), 0.3, 60, 1.0, torch.from_numpy(np.zeros(50, np.int8)).to(dev))
    np.testing.assert_allclose(out.cpu().numpy(), np.sign(v) * np.minimum(np.abs(v) / 1.3, 1.0), rtol=1e-14)
    # |J1| > k is rejected
    st = np.zeros(50, np.int8)
    st[:4] = oracle.ONE
    with pytest.raises(pr.PrError):
        pr.prox(torch.from_numpy(v).to(dev), 0.3, 3, 2.0, torch.from_numpy(st).to(dev))


@pytest.mark.parametrize("i", range(0, 56, 2))
def test_regularizer_matches_oracle(dev, i):
    import torch
    pr = _pr()
    v, rho, k, M, st = _prox_case(i)
    assert np.sum(st == oracle.ONE) <= k   # the generator draws |J1| <= k
    beta = oracle.prox_g(v, rho, k, M, st)   # a point of dom g_N
    beta[st == oracle.ZERO] = 0.0
    alpha = np.random.default_rng(i).standard_normal(v.size) * 3.0
    tst = torch.from_numpy(st).to(dev)
    g_gpu, gs_gpu = pr.regularizer(torch.from_numpy(beta).to(dev), torch.from_numpy(alpha).to(dev), k, M, tst)
    g_orc = oracle.g(beta, k, st) if oracle.in_dom(beta, k, M, st) else math.inf
    gs_orc = oracle.gstar(alpha, k, M, st)
    assert (g_gpu == g_orc) or abs(g_gpu - g_orc) <= 1e-12 * max(1.0, abs(g_orc))
    assert abs(gs_gpu - gs_orc) <= 1e-12 * max(1.0, abs(gs_orc))


def test_regularizer_worked_examples(dev):
    """Figure 3 worked examples: g(1.4, 0.6; k=1) = 2 and g(0.6, 1.2, 1.2; k=2) = 2.25."""
    import torch
    pr = _pr()
    g1, _ = pr.regularizer(torch.tensor([1.4, 0.6], dtype=torch.float64, device=dev), None, 1, 2.0,
                           torch.zeros(2, dtype=torch.int8, device=dev))
    g2, _ = pr.regularizer(torch.tensor([0.6, 1.2, 1.2], dtype=torch.float64, device=dev), None, 2, 1.5,
                           torch.zeros(3, dtype=torch.int8, device=dev))
    assert abs(g1 - 2.0) <= 1e-15 and abs(g2 - 2.25) <= 1e-15
    # off the domain (||beta||_1 > M k) the value is +inf
    g3, _ = pr.regularizer(torch.tensor([1.4, 0.6], dtype=torch.float64, device=dev), None, 1, 1.5,
                           torch.zeros(2, dtype=torch.int8, device=dev))
    assert g3 == math.inf


def _ctx_for(dev, Xcm, y, loss=0):
    import torch
    pr = _pr()
    if Xcm.dtype == np.uint16:
        X = torch.from_numpy(Xcm.view(np.int16)).to(dev).view(torch.bfloat16)
    else:
        X = torch.from_numpy(Xcm).to(dev)
    return pr.Context(X, torch.from_numpy(y).to(dev), loss)


@pytest.mark.parametrize("storage,n,p", [("f64", 500, 200), ("f64", 2, 1), ("f32", 1028, 37),
                                         ("f32", 4096, 1031), ("bf16", 1032, 77), ("bf16", 16384, 64),
                                         ("f32", 260, 10241), ("f64", 64, 16390), ("bf16", 520, 20483),
                                         ("f32", 128, 41000)])
def test_gemv_and_gemv_t_match_oracle(dev, storage, n, p):
    """Dense forward and transposed products element by element against the
    oracle's; p past 10240 and 20480 runs the transposed kernel with 4 and 8
    columns per wave, ragged against the workgroup's columns."""
    import torch
    inst = make_instance(n=n, p=p, corr=0.6, k_true=min(3, p), snr=5.0, loss=0, seed=7, storage=storage)
    ctx = _ctx_for(dev, inst.Xcm, inst.y)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(p)
    r = rng.standard_normal(n)
    u = ctx.gemv(torch.from_numpy(b).to(dev)).cpu().numpy()
    h = ctx.gemv_t(torch.from_numpy(r).to(dev)).cpu().numpy()
    X64 = inst.X64()
    u_ref = oracle.matvec(inst.Xcm, b)
    h_ref = oracle.rmatvec(inst.Xcm, r)
    # both sides sum exact FP64 products; only the summation order differs
    bound_u = 1e-13 * (np.abs(X64).T @ np.abs(b)) + 1e-300
    bound_h = 1e-13 * (np.abs(X64) @ np.abs(r)) + 1e-300
    assert np.all(np.abs(u - u_ref) <= bound_u)
    assert np.all(np.abs(h - h_ref) <= bound_h)
    ctx.close()


@pytest.mark.parametrize("storage,n,p", [("f32", 1028, 37), ("f32", 4096, 1031), ("f32", 200, 9), ("f64", 770, 65),
                                         ("f64", 2, 1), ("bf16", 1032, 77), ("bf16", 16384, 64), ("f32", 32768, 100),
                                         ("f32", 520, 6001), ("f64", 130, 9007), ("bf16", 1032, 16390)])
def test_gemv_t2_matches_oracle(dev, storage, n, p):
    """The two-right-hand-side transposed product (the logistic iteration's
    X^T [zeta, grad F]; 2, 4 or 8 columns per wave as p grows past 4096 and
    8192): both outputs element by element against the oracle's products, n
    ragged against the row step and p against the workgroup's columns."""
    import torch
    inst = make_instance(n=n, p=p, corr=0.6, k_true=min(3, p), snr=5.0, loss=1, seed=9, storage=storage)
    ctx = _ctx_for(dev, inst.Xcm, inst.y, loss=1)
    rng = np.random.default_rng(5)
    r1 = rng.standard_normal(n)
    r2 = rng.standard_normal(n) * 1e-3
    h1, h2 = ctx.gemv_t2(torch.from_numpy(r1).to(dev), torch.from_numpy(r2).to(dev))
    X64 = inst.X64()
    for h, r in ((h1.cpu().numpy(), r1), (h2.cpu().numpy(), r2)):
        ref = oracle.rmatvec(inst.Xcm, r)
        bound = 1e-13 * (np.abs(X64) @ np.abs(r)) + 1e-300
        assert np.all(np.abs(h - ref) <= bound)
    ctx.close()


def test_time_read_reads_only_and_rejects_bad_arguments(dev):
    """pr_time_read (the streaming-read rate the HBM-bound kernels are
    compared with): a positive time on both unroll forms and on grids whose
    stride leaves a ragged tail, the buffer unchanged, a read of 1 GiB no
    faster than 10 TB/s (a kernel whose loads were dropped), and PR_EINVAL before
    any launch for a length that is not a multiple of 16 bytes, an unaligned
    buffer, another unroll, an empty grid and zero repetitions."""
    import ctypes
    import torch
    import paper_2603_01306_amd as pr
    buf = torch.arange(1 << 20, dtype=torch.float32, device=dev)   # 4 MiB
    ref = buf.clone()
    for blocks, unroll in ((1, 1), (7, 4), (4096, 1), (3, 1)):
        assert pr.time_read(buf, blocks, unroll, reps=2) > 0.0
    torch.cuda.synchronize()
    assert torch.equal(buf, ref)
    # the loads are really issued: 1 GiB (4x the last-level cache) cannot be
    # read faster than 10 TB/s, above the HBM peak
    big = torch.zeros(1 << 28, dtype=torch.float32, device=dev)
    assert pr.time_read(big, 2048, 1, reps=3) >= (1 << 30) / 10e12 * 1e3
    del big
    lib = pr.load()
    ms = ctypes.c_double()
    base = buf.data_ptr()
    for args in ((base, 24, 1, 1, 1), (base + 4, 16, 1, 1, 1), (base, 16, 1, 3, 1), (base, 16, 0, 1, 1),
                 (base, 16, 1, 1, 0), (None, 16, 1, 1, 1)):
        ptr = ctypes.c_void_p(args[0]) if args[0] is not None else None
        assert lib.pr_time_read(ptr, args[1], args[2], args[3], args[4], None, ctypes.byref(ms)) == -1, args


@pytest.mark.parametrize("n,p,corr,storage", [(2048, 512, 0.9, "f32"), (64, 1000, 0.5, "f64"), (300, 1, 0.0, "f64"),
                                               (1000, 3, 0.99, "f64"), (4096, 2048, 0.5, "bf16")])
def test_norm2_matches_exact_eigenvalue(dev, n, p, corr, storage):
    """||X||_2^2 of the context (Lanczos on X^T X) against the largest
    eigenvalue of the smaller Gram matrix by a dense symmetric eigensolver:
    tall, wide (rank n < p), one column, and a few strongly correlated
    columns (the recurrence breaks down after p steps)."""
    inst = make_instance(n=n, p=p, corr=corr, k_true=1, snr=5.0, loss=0, seed=2, storage=storage)
    ctx = _ctx_for(dev, inst.Xcm, inst.y)
    X = inst.X64()
    lam = np.linalg.eigvalsh(X @ X.T if p <= n else X.T @ X).max()
    assert abs(ctx.norm2() - lam) <= 1e-10 * lam
    ctx.close()


@pytest.mark.parametrize("n,q", [(300, 1), (400, 50), (2048, 700)])
def test_norm2_of_mirrored_design(dev, n, q):
    """X = [A, -A]: every eigenvector of X^T X with a nonzero eigenvalue is
    (v, -v), orthogonal to the all-ones direction, so a recurrence started
    there sees only the zero eigenvalue.  ||X||_2^2 = 2 ||A||_2^2 exactly."""
    import torch
    pr = _pr()
    inst = make_instance(n=n, p=q, corr=0.5, k_true=1, snr=5.0, loss=0, seed=4, storage="f64")
    Xcm = np.ascontiguousarray(np.concatenate([inst.Xcm, -inst.Xcm], axis=0))
    ctx = pr.Context(torch.from_numpy(Xcm).to(dev), torch.from_numpy(inst.y).to(dev), 0)
    A = inst.X64()
    lam = 2.0 * np.linalg.eigvalsh(A @ A.T if q <= n else A.T @ A).max()
    assert abs(ctx.norm2() - lam) <= 1e-10 * lam
    ctx.close()


@pytest.mark.parametrize("p", [100, 6400, 102400])
def test_prox_and_g_at_microbenchmark_shapes(dev, p):
    """The paper's subroutine benchmark: gamma ~ N(0, I_p), root node, k = 10,
    M = 1, rho = 1; prox within 1e-12 of Algorithm 2 + Moreau (oracle) and
    g_N at beta = prox(gamma) within 1e-12 of Algorithm 1 (oracle)."""
    import torch
    import paper_2603_01306_amd as pr
    gamma = np.random.default_rng(p).standard_normal(p)
    st = torch.zeros(p, dtype=torch.int8, device=dev)
    out, ms_prox, ms_g = pr.time_prox(torch.from_numpy(gamma).to(dev), 1.0, 10, 1.0, st, reps=2)
    beta = out.cpu().numpy()
    ref = oracle.prox_g(gamma, 1.0, 10, 1.0)
    assert np.max(np.abs(beta - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    g_gpu, _ = pr.regularizer(out, None, 10, 1.0, st)
    g_ref = oracle.g(ref, 10)
    assert abs(g_gpu - g_ref) <= 1e-12 * max(1.0, abs(g_ref))
    assert ms_prox > 0 and ms_g > 0
