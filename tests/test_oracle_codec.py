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


# ------------------------------------------------------------------ golden --
# A record written bit by bit from the format description, whose inverse
# transform overflows 32 bits; the expected samples were worked out by hand
# (tests/golden/codec_wrap_record.json holds the bit segments and the
# derivation).  It pins the decoder's 32-bit wrapping inverse-transform rule.

def _golden():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "codec_wrap_record.json")
    with open(path) as fh:
        return json.load(fh)


def _pack_bits(segments, nbits):
    bits = []
    for seg in segments:
        bits += [int(ch) for ch in seg["bits"]] * int(seg.get("repeat", 1))
    assert len(bits) <= nbits
    words = np.zeros(nbits // 32, np.uint32)
    for i, b in enumerate(bits):
        if b:
            words[i >> 5] |= np.uint32(1 << (i & 31))
    return words, len(bits)


def test_golden_record_bits_match_their_segments():
    g = _golden()
    words, used = _pack_bits(g["bit_segments"], 64 * g["rate_bits"])
    assert used == 167
    assert [int(w, 16) for w in g["record_words_hex"]] == [int(w) for w in words]


def test_golden_record_wraps_in_32_bits():
    g = _golden()
    rec = np.array([int(w, 16) for w in g["record_words_hex"]], np.uint32)
    out = oracle.decode_block(rec.view(np.uint8), g["rate_bits"])
    want = np.array(g["expected_values"], np.float32)
    assert np.array_equal(out, want), np.nonzero(out != want)
    # the integers before scaling, as derived by hand (e = 0: value = q * 2^-27)
    q = np.array(g["expected_q"], np.int64)
    assert np.array_equal((q.astype(np.float64) * 2.0 ** -27).astype(np.float32), want)
    # the corner the wrap decides: -12 with the 32-bit rule, +20 without it
    assert out.reshape(4, 4, 4)[3, 3, 3] == np.float32(-12.0)


# -------------------------------------------------------------- truncation --
# Fixed rate means the record of block b is the first 64R bits of the
# embedded code.  These pin where the decoder stops and that it uses every
# bit up to there:
#   - the encoder's rate-R record is the first 64R bits of its rate-16 record
#     (embedded coding), so encoder and decoder cannot share an off-by-one at
#     the budget without this failing;
#   - the decoder reads nothing past 64R bits (changing the next record
#     changes nothing) and does read bit 64R-1 (flipping it changes the output
#     of some blocks);
#   - a block whose complete code fits in 64R bits decodes at rate R to the
#     block-floating-point quantisation of its values, computed here with
#     numpy from the format's definition (frexp exponent, truncation to 27
#     fraction bits).

def _bits(words):
    w = np.asarray(words, np.uint32)
    return ((w[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1).astype(np.uint8).reshape(-1)


def _blocks(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        kind = i % 5
        if kind == 4:
            # constant blocks of a few significant bits: codes short enough for rate 1
            v = np.full(64, float(rng.choice([1, 3, 5, -7, -1])) * 2.0 ** int(rng.integers(-20, 20)))
            v[int(rng.integers(0, 64))] *= float(rng.choice([1.0, 1.0, 0.5]))
        elif kind == 0:
            v = rng.standard_normal(64)
        elif kind == 1:
            v = np.cumsum(rng.standard_normal(64)) * 0.1 + 3.0
        elif kind == 2:
            v = np.zeros(64)
            idx = rng.choice(64, rng.integers(1, 6), replace=False)
            v[idx] = rng.integers(-6, 7, len(idx)) * 0.125
        else:
            v = np.sin(np.arange(64) * rng.uniform(0.05, 0.5)) * 10.0 ** rng.uniform(-3, 3)
        out.append(v.astype(np.float32))
    return out


@pytest.mark.parametrize("rate", [1, 2, 3, 4, 5, 6, 7, 8])
def test_rate_r_record_is_prefix_of_rate16_record(rate):
    for v in _blocks(100 + rate, 64):
        r16 = _bits(np.frombuffer(volgen.encode_block(v, 16).tobytes(), np.uint32))
        rr = _bits(np.frombuffer(volgen.encode_block(v, rate).tobytes(), np.uint32))
        assert len(rr) == 64 * rate
        assert np.array_equal(rr, r16[:64 * rate])


@pytest.mark.parametrize("rate", [1, 2, 4, 8])
def test_decoder_stops_exactly_at_the_budget(rate):
    nwords = 2 * rate
    changed = 0
    rng = np.random.default_rng(rate)
    for v in _blocks(200 + rate, 96):
        rec = np.frombuffer(volgen.encode_block(v, rate).tobytes(), np.uint32).copy()
        base = oracle.decode_block(rec.view(np.uint8), rate)
        # the next record's bits: zeros or random ones, never read
        tail = rng.integers(0, 2**32, nwords, dtype=np.uint64).astype(np.uint32)
        two = np.concatenate([rec, tail])
        s = two.view(np.uint8)
        dec = oracle.decode_blocks(s, (8, 4, 4), rate, np.array([0], np.uint32))[0]
        assert np.array_equal(dec, base)
        # the last bit of the record is read: flip it
        flip = rec.copy()
        flip[-1] ^= np.uint32(1 << 31)
        out = oracle.decode_block(flip.view(np.uint8), rate)
        changed += not np.array_equal(out, base)
    assert changed >= 4, changed   # a decoder stopping one bit early changes none


def _quantised(v):
    v = v.astype(np.float32)
    m = float(np.max(np.abs(v.astype(np.float64))))
    if m == 0.0:
        return np.zeros(64, np.float32)
    e = max(np.frexp(m)[1], -127)
    q = np.trunc(v.astype(np.float64) * 2.0 ** (27 - e))
    return (q * 2.0 ** (e - 27)).astype(np.float32)


@pytest.mark.parametrize("rate", [1, 2, 3, 4, 6, 8])
def test_complete_code_within_budget_decodes_to_the_quantisation(rate):
    fits = 0
    for v in _blocks(300 + rate, 200):
        r16 = _bits(np.frombuffer(volgen.encode_block(v, 16).tobytes(), np.uint32))
        # a rate-16 code that ended well before its budget and needs no bit
        # past 64R: the whole code fits in the rate-R record
        if r16[64 * rate:].any() or r16[512:].any():
            continue
        rec = volgen.encode_block(v, rate)
        out = oracle.decode_block(rec, rate)
        assert np.array_equal(out, _quantised(v)), (rate, np.nonzero(out != _quantised(v)))
        fits += 1
    assert fits >= 10, fits
