"""za_rhs_noalloc, the allocation-free right-hand side, against za_rhs.

Both run the same kernels; the allocation-free call keeps the wave-speed
reduction in a fixed device array instead of a context's workspace, so the
results must be equal bit for bit.  Two calls in a row, the second on a
smaller grid (the array keeps the first call's contents), in 2D and 1D, one
call on a non-default stream, and the argument checks.  Collected last (it
is named so), and it passes alone in a fresh process as well.
"""
import ctypes as C

import pytest

from paper_2603_26272_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


def ctx_rhs(P, q):
    from paper_2603_26272_amd.za import Context
    with Context(P) as ctx:
        return ctx.rhs(q)


def test_noalloc_rhs_equals_context_rhs_2d(dev):
    from paper_2603_26272_amd.za import rhs_noalloc
    for seed, n, ny in ((0, 512, 384), (1, 130, 67)):      # the second call is smaller
        P, q0 = W.quadrants_2d(seed, n, ny)
        q = torch.from_numpy(q0).to(dev)
        got = rhs_noalloc(P, q)
        ref = ctx_rhs(P, q)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (seed, n, ny)


def test_noalloc_rhs_equals_context_rhs_1d(dev):
    from paper_2603_26272_amd.za import rhs_noalloc
    for seed, n in ((2, 4096), (3, 300)):
        P, q0 = W.riemann_1d(seed, n)
        q = torch.from_numpy(q0).to(dev)
        got = rhs_noalloc(P, q)
        ref = ctx_rhs(P, q)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (seed, n)


def test_noalloc_rhs_on_a_side_stream(dev):
    from paper_2603_26272_amd.za import rhs_noalloc
    P, q0 = W.quadrants_2d(4, 96, 80)
    q = torch.from_numpy(q0).to(dev)
    ref = ctx_rhs(P, q)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got = rhs_noalloc(P, q, stream=s)
    s.synchronize()
    assert torch.equal(got, ref)


def test_noalloc_rhs_rejects_bad_arguments(dev):
    from paper_2603_26272_amd import za
    from paper_2603_26272_amd.problem import Problem
    P, q0 = W.quadrants_2d(4, 16, 16)
    q = torch.from_numpy(q0).to(dev)
    f = za.lib().za_rhs_noalloc
    qp = C.c_void_p(q.data_ptr())
    z = za.ZaProblem.from_problem(Problem(dim=3))
    out = torch.empty_like(q)
    assert f(C.byref(z), qp, C.c_void_p(out.data_ptr()), None) == za.ZA_ERR_ARG     # invalid problem
    z = za.ZaProblem.from_problem(P)
    assert f(C.byref(z), qp, qp, None) == za.ZA_ERR_ARG                              # q == rhs
    assert f(C.byref(z), None, C.c_void_p(out.data_ptr()), None) == za.ZA_ERR_ARG    # NULL q
