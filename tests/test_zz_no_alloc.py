"""mst_build_noalloc: the allocation-free entry point, through the C ABI.

It must give exactly the tree mst_build gives (same kernels, the library's
fixed device scratch in place of the caller's workspace), also on a second
call in a row with a smaller input, whose scratch still holds the first
call's contents; inputs too large for the scratch are refused before any
device work.
"""
import ctypes

import numpy as np
import pytest

from paper_1402_3789_amd import _native as N
import paper_1402_3789_amd as nnm
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    t = pytest.importorskip("torch")
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _noalloc(torch, X, prec):
    """Call mst_build_noalloc directly through ctypes; returns the raw edge
    bytes and the report."""
    n, d = X.shape
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0")
    edges = torch.full((max(n - 1, 1), 3), float("nan"), dtype=torch.float64, device="cuda:0")
    o = nnm.options(prec)
    rep = N.Report()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = N.lib().mst_build_noalloc(ctypes.c_void_p(Xd.data_ptr()), n, d, d, ctypes.byref(o),
                                     ctypes.c_void_p(edges.data_ptr()), stream, ctypes.byref(rep))
    torch.cuda.synchronize()
    return code, edges[: n - 1].cpu().numpy().view(np.uint8).reshape(-1), rep


def _with_workspace(torch, X, prec):
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0")
    tree = nnm.mst_build(Xd, precision=prec)
    torch.cuda.synchronize()
    return tree.host_bytes()


@pytest.mark.parametrize("prec", ["auto", "fp32"])
def test_noalloc_matches_workspace_entry_point_twice(torch, prec):
    big, _ = W.mixture64(3, n=20000, d=25)
    small, _ = W.blobs8(4, n=3001, d=8)
    for case, X in (("20000x25", big), ("3001x8 after 20000x25", small)):
        print(f"[no_alloc] {prec} {case}", flush=True)
        code, got, rep = _noalloc(torch, X, prec)
        assert code == 0, f"{case}: {N.strerror(code)}"
        want = _with_workspace(torch, X, prec)
        assert got.shape == want.shape
        assert np.array_equal(got, want), f"{prec} {case}: tree differs from mst_build"
        assert rep.rounds >= 1 and rep.ms_candidates == 0.0


def test_noalloc_public_binding(torch):
    X, _ = W.blobs8(5, n=1500, d=8)
    Xd = torch.from_numpy(X).to("cuda:0")
    t1 = nnm.mst_build_noalloc(Xd)
    t2 = nnm.mst_build(Xd)
    torch.cuda.synchronize()
    assert np.array_equal(t1.host_bytes(), t2.host_bytes())


def test_noalloc_refuses_inputs_beyond_the_scratch(torch):
    n, d = 300_000, 25
    nb = ctypes.c_size_t(0)
    o = nnm.options()
    assert N.lib().mst_workspace_size(n, d, ctypes.byref(o), ctypes.byref(nb)) == 0
    assert nb.value > N.NOALLOC_SCRATCH_BYTES
    Xd = torch.zeros((n, d), dtype=torch.float32, device="cuda:0")
    edges = torch.empty((n - 1, 3), dtype=torch.float64, device="cuda:0")
    code = N.lib().mst_build_noalloc(ctypes.c_void_p(Xd.data_ptr()), n, d, d, ctypes.byref(o),
                                     ctypes.c_void_p(edges.data_ptr()), None, None)
    assert code == N.NNM_ETOOLARGE
    assert "scratch" in N.strerror(code)
    # the refused call left the scratch usable
    X, _ = W.blobs8(6, n=700, d=8)
    code, got, _ = _noalloc(torch, X, "auto")
    assert code == 0 and np.array_equal(got, _with_workspace(torch, X, "auto"))
