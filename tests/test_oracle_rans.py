"""Pins for the interleaved rANS oracle: hand vectors, round trips, the
per-symbol definition vs the lane-parallel form, integrity, code length."""
import numpy as np
import pytest

from oracle import entropy, rans

FREQ, CUM = entropy.cdf_tables()


def _states(seg):
    return np.frombuffer(seg[:128], "<u4")


def test_hand_vector_one_symbol_no_word():
    freq = np.array([[1 << 15, 1 << 15]])
    cum = np.array([[0, 1 << 15]])
    seg = rans.encode_segment_ref([1], [0], freq, cum)
    st = _states(seg)
    assert st[0] == (1 << 17) + (1 << 15)
    assert np.all(st[1:] == 1 << 16)
    assert len(seg) == 128
    assert rans.decode_segment_ref(seg, [0], freq, cum) == [1]
    assert rans.encode([1], [0], freq, cum, 32)[0] == seg


def test_hand_vector_two_symbols_one_word():
    # Table row: f = (1, 65535), cum = (0, 1).  Lane 0 codes symbol 1 at step 0
    # and symbol 0 at step 1; lanes 1..31 code symbol 1 at step 0.
    # Lane 0 (encoded backwards): x = 2^16 >= 1 * 2^16, so push word 0 and x = 1;
    # C(0, 1) = 1 * 65536 + 0 + 0 = 65536; then C(1, 65536) = 1 * 65536 + 1 + 1 = 65538.
    # Lanes 1..31: C(1, 65536) = 65538 with no push.
    freq = np.array([[1, 65535]])
    cum = np.array([[0, 1]])
    sym = [1] * 32 + [0]
    idx = [0] * 33
    seg = rans.encode_segment_ref(sym, idx, freq, cum)
    assert np.all(_states(seg) == 65538)
    assert len(seg) == 128 + 4  # one word plus the alignment pad
    assert np.all(np.frombuffer(seg[128:], "<u2") == 0)
    assert rans.decode_segment_ref(seg, idx, freq, cum) == sym
    assert rans.encode(sym, idx, freq, cum, 64)[0] == seg


def test_hand_vector_renormalises_on_the_boundary():
    # x = 2^16 equals f * 2^16 for f = 1: the word must be pushed *before* coding,
    # otherwise the state would leave 32 bits (2^16 * 2^16 = 2^32).
    freq = np.array([[1, 65535]])
    cum = np.array([[0, 1]])
    seg = rans.encode_segment_ref([0], [0], freq, cum)
    assert _states(seg)[0] == 65536 and len(seg) == 132
    assert rans.encode([0], [0], freq, cum, 32)[0] == seg
    assert rans.decode_segment_ref(seg, [0], freq, cum) == [0]


@pytest.mark.parametrize("n,seg", [(1, 32), (31, 32), (32, 32), (33, 64), (1000, 256), (4097, 1024)])
def test_vector_form_matches_definition(n, seg):
    rng = np.random.default_rng(n)
    idx = rng.integers(0, 64, n)
    sym = np.clip(np.rint(rng.standard_normal(n) * entropy.scales()[idx]), -32, 32).astype(int) + 32
    vec = rans.encode(sym, idx, FREQ, CUM, seg)
    ref = [rans.encode_segment_ref(sym[a:a + seg], idx[a:a + seg], FREQ, CUM)
           for a in range(0, n, seg)]
    assert vec == ref
    back = rans.decode(vec, idx, FREQ, CUM, seg)
    np.testing.assert_array_equal(back, sym)
    for a, s in zip(range(0, n, seg), ref):
        assert rans.decode_segment_ref(s, idx[a:a + seg], FREQ, CUM) == list(sym[a:a + seg])


@pytest.mark.parametrize("kind", ["tails", "centre", "uniform_rows", "mixed"])
def test_round_trip_adversarial(kind):
    rng = np.random.default_rng(5)
    n = 5000
    if kind == "tails":      # f = 1 symbols under the narrowest table: one word each
        idx = np.zeros(n, int)
        sym = rng.choice([0, 64], n)
    elif kind == "centre":   # 0.0014 bits each
        idx = np.zeros(n, int)
        sym = np.full(n, 32)
    elif kind == "uniform_rows":
        idx = np.full(n, 63)
        sym = rng.integers(0, 65, n)
    else:
        idx = rng.integers(0, 64, n)
        sym = rng.integers(0, 65, n)
    segs = rans.encode(sym, idx, FREQ, CUM, 1024)
    np.testing.assert_array_equal(rans.decode(segs, idx, FREQ, CUM, 1024), sym)
    if kind == "tails":
        assert all(len(s) >= 128 + 2 * 1000 for s in segs[:-1])


def test_code_length_bound():
    rng = np.random.default_rng(6)
    n = 1 << 18
    idx = rng.integers(0, 64, n)
    # draw symbols from the quantised distributions themselves
    u = rng.integers(0, 65536, n)
    sym = np.array([np.searchsorted(CUM[k], v, side="right") - 1 for k, v in zip(idx, u)])
    ideal = entropy.ideal_bits(sym, idx, FREQ)
    for seg in (1 << 12, 1 << 15, 1 << 18):
        segs = rans.encode(sym, idx, FREQ, CUM, seg)
        bits = 8 * sum(len(s) for s in segs)
        assert 0 <= bits - ideal <= 0.005 * ideal + 32 * 32 * len(segs)
    # one segment: the literal bound holds
    assert bits - ideal <= 0.005 * ideal


def test_corruption_is_detected():
    rng = np.random.default_rng(7)
    n = 4096
    idx = rng.integers(0, 64, n)
    sym = np.clip(np.rint(rng.standard_normal(n) * 3), -32, 32).astype(int) + 32
    seg = rans.encode(sym, idx, FREQ, CUM, n)[0]
    with pytest.raises(rans.CorruptStream):
        rans.decode([seg[:-4]], idx, FREQ, CUM, n)
    with pytest.raises(rans.CorruptStream):
        rans.decode([seg + b"\0\0\0\0"], idx, FREQ, CUM, n)
    for pos in (0, 3, 64, 127, 200, len(seg) - 6):
        bad = bytearray(seg)
        bad[pos] ^= 0x5A
        with pytest.raises(rans.CorruptStream):
            rans.decode([bytes(bad)], idx, FREQ, CUM, n)
