"""Pins of the oracle's block decoder (fixed-rate block decompression, Sec. 3.5).

The codec is project-defined (format version 1, written out in volgen.c), so
beyond the properties below parity is unpinned against any external stream:
no zfp streams exist here.  What pins the oracle decoder is the independent
encoder (separate code doing the inverse operations) and mathematics:
  - raw mode is the identity, bit for bit;
  - constant blocks decode exactly at every rate >= 2 (block-floating-point
    quantisation of one float is exact and the transform keeps only the DC);
  - blocks whose values are multiples of a coarse power of two decode exactly
    at rate 16, which needs every inverse-transform index, the coefficient
    order and the plane coder right;
  - RMS error falls strictly with the rate;
  - single-block and whole-volume decodes agree.
"""
import numpy as np
import pytest

import oracle
import volgen


def _rt(v64, rate):
    rec = volgen.encode_block(v64, rate)
    return oracle.decode_block(rec, rate)


def test_raw_mode_identity_bitwise():
    rng = np.random.default_rng(11)
    v = rng.standard_normal(64).astype(np.float32) * np.float32(1e3)
    v[0] = np.float32(-0.0)
    v[1] = np.float32(1e-45)          # smallest subnormal
    v[2] = np.float32(3.4e38)
    out = _rt(v, 32)
    assert out.tobytes() == v.tobytes()


@pytest.mark.parametrize("rate", [2, 4, 8, 16])
@pytest.mark.parametrize("val", [0.5, -0.7, 1.0, 123.456, -3.0e-39, 1.0e-45, 2.5e37, 0.0])
def test_constant_block_exact(rate, val):
    v = np.full(64, val, np.float32)
    out = _rt(v, rate)
    assert np.array_equal(out, v), (rate, val, out[:4])


def test_zero_block_decodes_to_positive_zero():
    out = _rt(np.full(64, -0.0, np.float32), 4)
    assert out.tobytes() == np.zeros(64, np.float32).tobytes()


@pytest.mark.parametrize("seed", range(8))
def test_dyadic_blocks_exact_at_rate16(seed):
    rng = np.random.default_rng(seed)
    v = (rng.integers(-1, 2, 64) * 0.5).astype(np.float32)
    if not np.any(v):
        v[5] = 0.5
    out = _rt(v, 16)
    assert np.array_equal(out, v), np.nonzero(out != v)


def test_single_sample_impulses_exact_at_rate16():
    # an impulse at every position exercises every inverse-transform path
    for i in range(64):
        v = np.zeros(64, np.float32)
        v[i] = -0.75 if i % 3 else 0.5
        out = _rt(v, 16)
        assert np.array_equal(out, v), i


def test_rms_falls_with_rate():
    vol = volgen.blobs(32, 32, 32, seed=5)
    errs = []
    for rate in (2, 4, 8, 16):
        s = volgen.encode(vol, rate)
        d = oracle.decode_volume(s, (32, 32, 32), rate)
        errs.append(float(np.sqrt(np.mean((d.astype(np.float64) - vol) ** 2))))
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    # rate 16 keeps ~ all of the 24-bit mantissa budget on a smooth field
    assert errs[-1] < 1e-5 * float(np.abs(vol).max())


def test_partial_blocks_and_bulk_equals_single():
    vol = volgen.blobs(13, 10, 7, seed=9)     # ragged edges on every axis
    for rate in (2, 8, 32):
        s = volgen.encode(vol, rate)
        assert s.nbytes == 4 * 3 * 2 * 8 * rate
        d = oracle.decode_volume(s, (13, 10, 7), rate)
        ids = np.arange(4 * 3 * 2, dtype=np.uint32)
        blk = oracle.decode_blocks(s, (13, 10, 7), rate, ids)
        for b in ids:
            bx, by, bz = b % 4, (b // 4) % 3, b // 12
            for k in range(4):
                for j in range(4):
                    for i in range(4):
                        x, y, z = 4 * bx + i, 4 * by + j, 4 * bz + k
                        if x < 13 and y < 10 and z < 7:
                            assert blk[b, i + 4 * j + 16 * k] == d[z, y, x]
        if rate == 32:
            assert np.array_equal(d, vol)


def test_stream_size_validation():
    vol = volgen.blobs(8, 8, 8, seed=1)
    s = volgen.encode(vol, 4)
    with pytest.raises(RuntimeError):
        oracle.decode_volume(s[:-1], (8, 8, 8), 4)
