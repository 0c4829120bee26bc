"""GPU parity of the foveal decoder (vrs_decode_fovea) and of the
combination (vrs_composite_frame) against the CPU reference: float32 MFMA
path within 1e-4, bfloat16 MFMA path within 2e-2 (both relative to the
output's largest magnitude), on uneven crop sizes across two views."""
import numpy as np
import pytest
import torch

import oracle
from paper_2410_17932_amd import api, synth

from gpu_helpers import dev

pytestmark = pytest.mark.gpu


def _setup(seed, widths, crops_spec, L, W=200, H=160, nv=2, bias=True):
    rng = np.random.default_rng(seed)
    dw = synth.decoder_weights(rng, widths, 4)
    if bias:
        dw["levels"] = [(w, rng.normal(0, 0.1, b.shape).astype(np.float32)) for w, b in dw["levels"]]
        dw["head"] = (dw["head"][0], rng.normal(0, 0.1, 3).astype(np.float32))
    views = [synth.pinhole(W, H, 150.0, (0.03 * i, 0, 0)) for i in range(nv)]
    crops = [synth.crop_at(v, gx, gy, s, W, H) for v, gx, gy, s in crops_spec]
    ci, _ = synth.crops_array(crops)
    P = oracle.pyramid_pixels(ci, L)
    pyr = rng.normal(size=(P, 4)).astype(np.float32)
    periph = rng.uniform(size=(nv, 3, H, W)).astype(np.float32)
    return dw, views, crops, ci, pyr, periph


@pytest.mark.parametrize("dtype,tol", [(api.VRS_F32, 1e-4), (api.VRS_BF16, 2e-2)])
@pytest.mark.parametrize("widths,L", [((8, 8), 4), ((16, 32, 64, 64), 4), ((16, 24), 3)])
def test_decoder_parity(dtype, tol, widths, L):
    spec = [(0, 60.0, 50.0, 64), (1, 120.0, 90.0, 96), (0, 150.0, 100.0, 32), (1, 10.0, 10.0, 128)]
    dw, views, crops, ci, pyr, periph = _setup(41, widths, spec, L)
    D = synth.views_dims(views)
    packed = synth.pack_decoder(dw)
    ref = oracle.decode(ci, L, 4, pyr.astype(np.float64), periph.astype(np.float64), D, widths,
                        packed.astype(np.float64))
    ws = api.DecoderWorkspace(widths, crops, dtype)
    out = api.decode_fovea(dev(pyr), L, dev(periph), views, crops, dev(packed), ws)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    scale = max(1.0, np.abs(ref).max())
    err = np.abs(got - ref).max() / scale
    print(f"decoder {widths} dtype={dtype} rel max err {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("mode", [api.BLEND_LINEAR, api.BLEND_PAPER])
@pytest.mark.parametrize("W", [180, 181])   # four pixels per thread, and one
def test_composite_parity(mode, W):
    rng = np.random.default_rng(5)
    H = 150
    views = [synth.pinhole(W, H, 150.0), synth.pinhole(W, H, 150.0, (0.06, 0, 0))]
    crops = [synth.crop_at(0, 60.3, 70.7, 64, W, H), synth.crop_at(0, 80.0, 80.0, 96, W, H),
             synth.crop_at(1, 170.0, 10.0, 32, W, H), synth.crop_at(1, 90.0, 75.0, 128, W, H)]
    ci, cf = synth.crops_array(crops)
    P = rng.uniform(size=(2, 3, H, W)).astype(np.float32)
    F = rng.uniform(size=sum(3 * c.size ** 2 for c in crops)).astype(np.float32)
    # smooth F a little so the edge term spans (0, 1)
    ref = oracle.composite(P.astype(np.float64), synth.views_dims(views), ci, cf,
                           F.astype(np.float64), mode=mode, ring=16.0, m=0.75, gamma=0.2)
    out = api.composite_frame(dev(P), dev(F), crops, mode=mode, ring=16.0)
    torch.cuda.synchronize()
    err = np.abs(out.cpu().numpy() - ref).max()
    assert err <= 1e-5, err


@pytest.mark.parametrize("mode", [api.BLEND_LINEAR, api.BLEND_PAPER])
@pytest.mark.parametrize("W", [180, 181])
def test_composite_in_place(mode, W):
    """Combination into the periphery image itself (only the pixels under the
    crops are touched, overlapping crops once each) equals the combination
    into a separate image bit for bit."""
    rng = np.random.default_rng(9)
    H = 150
    crops = [synth.crop_at(0, 60.3, 70.7, 64, W, H), synth.crop_at(0, 80.0, 80.0, 96, W, H),
             synth.crop_at(0, 70.0, 60.0, 32, W, H), synth.crop_at(1, 170.0, 10.0, 32, W, H),
             synth.crop_at(1, 90.0, 75.0, 128, W, H)]
    P = dev(rng.uniform(size=(2, 3, H, W)).astype(np.float32))
    F = dev(rng.uniform(size=sum(3 * c.size ** 2 for c in crops)).astype(np.float32))
    sep = api.composite_frame(P, F, crops, mode=mode, ring=16.0)
    io = P.clone()
    api.composite_frame(io, F, crops, mode=mode, ring=16.0, out=io)
    torch.cuda.synchronize()
    assert torch.equal(io, sep)
