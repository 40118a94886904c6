"""The allocation-free candidate sampler (rf_sample_cells_noalloc) through the
C ABI against rf_sample_cells with a caller workspace: bit-exact cell indices
on two calls in a row, the second with fewer cells, and the size limit."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _reference(L, scores, draws):
    """rf_sample_cells with a workspace of the size rf_sample_workspace asks for."""
    import torch

    n, k = scores.numel(), draws.numel()
    nbytes = ctypes.c_size_t()
    assert L.lib().rf_sample_workspace(n, ctypes.byref(nbytes)) == 0
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")
    out = torch.full((k,), -7, dtype=torch.int32, device="cuda")
    assert L.lib().rf_sample_cells(scores.data_ptr(), n, draws.data_ptr(), k, out.data_ptr(), ws.data_ptr(),
                                   ws.numel(), _stream()) == 0
    return out


def test_noalloc_sampler_matches_workspace_sampler():
    import torch

    from paper_2502_01157_amd import _lib as L

    lib = L.lib()
    for n, k, seed in ((1_000_003, 200_000, 1), (70_001, 30_000, 2)):
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        scores = torch.rand(n, device="cuda", generator=g) ** 3
        scores[torch.rand(n, device="cuda", generator=g) < 0.3] = 0.0  # cells that are never drawn
        draws = torch.rand(k, device="cuda", generator=g)
        ref = _reference(L, scores, draws)
        out = torch.full((k,), -7, dtype=torch.int32, device="cuda")
        print(f"noalloc sampler: n={n} draws={k} seed={seed}", flush=True)
        assert lib.rf_sample_cells_noalloc(scores.data_ptr(), n, draws.data_ptr(), k, out.data_ptr(),
                                           _stream()) == L.RF_OK
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        o = out.cpu().numpy()
        assert o.min() >= 0 and o.max() < n
        assert np.all(scores.cpu().numpy()[o] > 0)
    # beyond the limit the call is refused on the host (nothing is launched)
    limit = 1 << 22
    assert lib.rf_sample_cells_noalloc(scores.data_ptr(), limit + 1, draws.data_ptr(), k, out.data_ptr(),
                                       _stream()) == 4  # RF_ERR_UNSUPPORTED
    assert b"limit" in lib.rf_last_error()
    assert lib.rf_sample_cells_noalloc(scores.data_ptr(), 0, draws.data_ptr(), k, out.data_ptr(),
                                       _stream()) == L.RF_ERR_INVALID_ARG
