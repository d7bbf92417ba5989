"""GPU: the allocation-free forward pass of the correction network (bem_mlp_forward_noalloc)
against the workspace entry point (bem_mlp_forward), through the C ABI.

Bar: the same kernels run on the same inputs, so the outputs are bitwise equal; two calls
in a row, the second with a smaller batch (the fixed scratch keeps the first call's
contents), for FP32 and BF16 products.  Sizes beyond the fixed scratch are refused on the
host before any launch.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

IN, HID, OUT = 99, 256, 2048


@pytest.fixture(scope="module")
def C():
    import paper_1906_00785_amd as B

    return B._bem


def _net(C, seed):
    nparams, _ = C.bem_mlp_sizes(IN, HID, OUT, 1)
    p = torch.empty(nparams, dtype=torch.float32, device="cuda")
    C.bem_mlp_init(IN, HID, OUT, seed, p.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return p


def _forward_ws(C, p, X, prec):
    st = torch.cuda.current_stream().cuda_stream
    _, nbytes = C.bem_mlp_sizes(IN, HID, OUT, X.shape[0])
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    Y = torch.empty(X.shape[0], OUT, dtype=torch.float32, device="cuda")
    C.bem_mlp_forward(IN, HID, OUT, X.shape[0], p.data_ptr(), X.data_ptr(), Y.data_ptr(), prec, ws.data_ptr(),
                      nbytes, st)
    return Y


def _forward_noalloc(C, p, X, prec):
    st = torch.cuda.current_stream().cuda_stream
    Y = torch.full((X.shape[0], OUT), float("nan"), dtype=torch.float32, device="cuda")
    C.bem_mlp_forward_noalloc(IN, HID, OUT, X.shape[0], p.data_ptr(), X.data_ptr(), Y.data_ptr(), prec, st)
    return Y


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_forward_matches_workspace_forward(C, prec):
    p = _net(C, 1906 + prec)
    for k, batch in enumerate((1089, 150)):  # the second call is smaller: stale scratch beyond it
        print(f"[no-alloc] precision {prec} call {k} batch {batch}", flush=True)
        X = torch.from_numpy(W.rng(4, 500 + 10 * prec + k).normal(size=(batch, IN)).astype(np.float32)).cuda()
        Yn = _forward_noalloc(C, p, X, prec)
        Yw = _forward_ws(C, p, X, prec)
        torch.cuda.synchronize()
        assert torch.isfinite(Yn).all()
        assert torch.equal(Yn, Yw), (prec, batch)


def test_noalloc_forward_refuses_oversized_batches(C):
    p = _net(C, 7)
    X = torch.zeros(1, IN, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    too_many = (32 << 20) // (8 * HID) + 1  # one row beyond the fixed scratch
    with pytest.raises(Exception) as e:
        C.bem_mlp_forward_noalloc(IN, HID, OUT, too_many, p.data_ptr(), X.data_ptr(), X.data_ptr(), 0, st)
    assert "scratch" in str(e.value)
    with pytest.raises(Exception):
        C.bem_mlp_forward_noalloc(IN, HID, OUT, 0, p.data_ptr(), X.data_ptr(), X.data_ptr(), 0, st)
