"""Exhaustive and long-stream checks of the generated operand on the GPU.

The entries of Omega must be bit-exact against the oracle (Sec. 6.3 generator;
the Box-Muller reading of the library's Omega definition).  Sampled blocks
cover only a few hundred thousand uniforms, so:

* the device's normal transform (sketch_normal_raw: the same inlined code the
  product kernels run) is compared bit for bit with the oracle's over every one
  of the 2^23 radius uniforms (even word) and every one of the 2^23 angle
  uniforms (odd word), each paired with several values of the other word;
* 2^25 consecutive entries of one Omega column (2^23 Philox calls, 2^24
  Box-Muller pairs) from sketch_gen_omega are compared bit for bit with the
  oracle's block, at a row offset past 2^32 so the counter's high word is live.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_20966_amd as sk

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _pairs_on_device(ev: np.ndarray, od: np.ndarray) -> np.ndarray:
    w = np.stack([ev, od], axis=1).astype(np.uint32)
    out = sk.sketch_normal_raw(torch.from_numpy(w.view(np.int32)).to(DEV))
    return out.cpu().numpy()


@pytest.mark.parametrize("fixed", [0x00000000, 0x5A3C9E00, 0xFFFFFFFF, 0x80000000])
def test_every_radius_uniform(fixed):
    """Even word over all 2^23 uniforms (the 9 discarded low bits vary too)."""
    x = np.arange(1 << 23, dtype=np.uint64)
    ev = ((x << 9) | ((x * 2654435761) & 0x1FF)).astype(np.uint32)
    od = np.full(ev.shape, fixed, dtype=np.uint32)
    got = _pairs_on_device(ev, od)
    zc, zs = oracle.normal_pairs(ev, od)
    assert np.array_equal(got[:, 0].view(np.uint32), zc.view(np.uint32))
    assert np.array_equal(got[:, 1].view(np.uint32), zs.view(np.uint32))


@pytest.mark.parametrize("fixed", [0x00000000, 0x12345600, 0xFFFFFFFF, 0x7FFFFE00])
def test_every_angle_uniform(fixed):
    """Odd word over all 2^23 uniforms: every quadrant and every reduced argument."""
    y = np.arange(1 << 23, dtype=np.uint64)
    od = ((y << 9) | ((y * 40503) & 0x1FF)).astype(np.uint32)
    ev = np.full(od.shape, fixed, dtype=np.uint32)
    got = _pairs_on_device(ev, od)
    zc, zs = oracle.normal_pairs(ev, od)
    assert np.array_equal(got[:, 0].view(np.uint32), zc.view(np.uint32))
    assert np.array_equal(got[:, 1].view(np.uint32), zs.view(np.uint32))


def test_long_column_stream_bit_exact():
    """2^25 consecutive rows of one column, starting past 2^32 rows (+ an unaligned
    start), against the oracle's block."""
    n = 1 << 25
    row0 = (1 << 34) + 3
    Om = sk.sketch_gen_omega(0xC0FFEE, row0, n, 7, 1, device=DEV).cpu().numpy()
    ref = oracle.omega_block(0xC0FFEE, row0, n, 7, 1)
    assert np.array_equal(Om.view(np.uint32), ref.view(np.uint32))
    # the stream is really N(0,1): a sanity check of the long column
    assert abs(float(ref.mean())) < 1e-3 and abs(float(ref.var()) - 1.0) < 2e-3
