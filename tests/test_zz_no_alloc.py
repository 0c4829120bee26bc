"""The allocation-free spatial order (vrs_spatial_order_noalloc, scratch in
a fixed device array of the library) against the workspace form
vrs_spatial_order, through the C-ABI: the same permutation bit for bit on
two calls in a row, the second with a smaller input (the array keeps the
first call's contents), and the size limit rejected on the host."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2410_17932_amd import api, synth

pytestmark = pytest.mark.gpu


def _points(seed, n):
    rng = np.random.default_rng(seed)
    pos = synth.points(rng, n, "uniform")["pos"]
    # exact duplicates too: the order of equal codes is the input order
    pos[:, n // 2: n // 2 + 50] = pos[:, :50]
    return torch.from_numpy(pos).cuda()


def _workspace_form(pos):
    n = pos.shape[1]
    size = api.lib().vrs_spatial_order_workspace_size(n)
    ws = torch.empty(size, dtype=torch.uint8, device="cuda")
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    code = api.lib().vrs_spatial_order(api.ptr(pos), n, api.ptr(perm), api.ptr(ws), size,
                                       api._stream())
    assert code == api.VRS_OK
    return perm


def _noalloc_form(pos):
    n = pos.shape[1]
    perm = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    code = api.lib().vrs_spatial_order_noalloc(api.ptr(pos), n, api.ptr(perm), api._stream())
    assert code == api.VRS_OK
    return perm


def test_noalloc_matches_workspace_form_twice():
    for seed, n in ((1, api.NOALLOC_MAX_POINTS), (2, 123_457)):
        pos = _points(seed, n)
        a = _noalloc_form(pos)
        b = _workspace_form(pos)
        torch.cuda.synchronize()
        assert torch.equal(a, b), f"n={n}"
        assert torch.equal(torch.sort(a.long())[0], torch.arange(n, device="cuda"))


def test_noalloc_rejects_beyond_its_limit():
    pos = torch.zeros((3, api.NOALLOC_MAX_POINTS + 1), device="cuda")
    perm = torch.empty(api.NOALLOC_MAX_POINTS + 1, dtype=torch.int32, device="cuda")
    code = api.lib().vrs_spatial_order_noalloc(api.ptr(pos), pos.shape[1], api.ptr(perm),
                                               api._stream())
    assert code == api.VRS_EINVAL
    assert api.lib().vrs_spatial_order_noalloc(None, 10, api.ptr(perm), api._stream()) == api.VRS_EINVAL
    assert api.lib().vrs_spatial_order_noalloc(api.ptr(pos), 0, api.ptr(perm),
                                               api._stream()) == api.VRS_EINVAL
