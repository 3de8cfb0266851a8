"""Interleaved 32-lane rANS over the quantised Gaussian tables.

Test infrastructure only (see the package docstring).

The paper codes r_hat with an arithmetic coder ("AE"/"AD" in Fig. 3) whose
type it does not name.  This oracle follows range asymmetric numeral systems
(Duda 2013, arXiv:1311.2540) with the interleaving of Giesen 2014
(arXiv:1402.3392), written from their mathematics:

  * state x in [L, 2^32) with L = 2^16, frequencies summing to M = 2^16, one
    16-bit word moved per renormalisation (at most one per symbol);
  * a segment of n symbols is spread over 32 lanes: symbol j belongs to lane
    j mod 32 at step floor(j / 32);
  * encoding runs backwards (last step first, lanes 31..0 within a step):
    if x >= f * 2^16 push the low 16 bits and shift; then
    x <- floor(x / f) * M + (x mod f) + c;
  * a segment is 32 little-endian u32 final states (lane 0..31), then the
    pushed words in pop order (last pushed first) as u16 LE, then one zero u16
    if needed to make the length a multiple of 4 bytes;
  * decoding runs forwards (step 0 first, lanes 0..31):
    slot = x mod M, s = the symbol with cum_s <= slot < cum_s + f_s,
    x <- f_s * floor(x / M) + slot - cum_s, and if x < L one word is shifted
    in; at the end every lane must be back at L and every word consumed.

``encode_segment_ref`` / ``decode_segment_ref`` are the per-symbol definition
in pure Python integers (small inputs).  ``encode`` / ``decode`` run the same
per-lane arithmetic for all lanes and segments at once with numpy uint64; a
test checks them against the per-symbol definition.  Pins: hand-computed
one- and two-symbol vectors, exact round trips, final states, the code-length
bound against sum(-log2 p).
"""
from __future__ import annotations

import numpy as np

LANES = 32
L = 1 << 16
PREC = 16
M = 1 << PREC
STATE_BYTES = 4 * LANES


class CorruptStream(ValueError):
    """The bit-stream does not decode to a consistent final state."""


# --------------------------------------------------------------------------
# Per-symbol definition (pure Python ints)
# --------------------------------------------------------------------------

def encode_segment_ref(sym, idx, freq, cum) -> bytes:
    n = len(sym)
    x = [L] * LANES
    pushed: list[int] = []
    nsteps = -(-n // LANES)
    for step in reversed(range(nsteps)):
        for lane in reversed(range(LANES)):
            j = step * LANES + lane
            if j >= n:
                continue
            f = int(freq[idx[j]][sym[j]])
            c = int(cum[idx[j]][sym[j]])
            if x[lane] >= (f << 16):
                pushed.append(x[lane] & 0xFFFF)
                x[lane] >>= 16
            x[lane] = (x[lane] // f) * M + (x[lane] % f) + c
    words = pushed[::-1]
    if len(words) % 2:
        words.append(0)
    out = bytearray()
    for v in x:
        out += int(v).to_bytes(4, "little")
    for w in words:
        out += int(w).to_bytes(2, "little")
    return bytes(out)


def decode_segment_ref(data: bytes, idx, freq, cum) -> list[int]:
    n = len(idx)
    if len(data) < STATE_BYTES or len(data) % 4:
        raise CorruptStream("segment too short or misaligned")
    x = [int.from_bytes(data[4 * i:4 * i + 4], "little") for i in range(LANES)]
    words = [int.from_bytes(data[i:i + 2], "little") for i in range(STATE_BYTES, len(data), 2)]
    pos = 0
    out = [0] * n
    nsteps = -(-n // LANES)
    for step in range(nsteps):
        for lane in range(LANES):
            j = step * LANES + lane
            if j >= n:
                continue
            k = int(idx[j])
            slot = x[lane] & (M - 1)
            s = 0
            while s + 1 < freq.shape[1] and int(cum[k][s + 1]) <= slot:
                s += 1
            x[lane] = int(freq[k][s]) * (x[lane] >> PREC) + slot - int(cum[k][s])
            if x[lane] < L:
                if pos >= len(words):
                    raise CorruptStream("ran out of words")
                x[lane] = (x[lane] << 16) | words[pos]
                pos += 1
            out[j] = s
    if any(v != L for v in x):
        raise CorruptStream("final state is not L")
    rest = len(words) - pos
    if rest not in (0, 1) or (rest == 1 and (words[pos] != 0 or pos % 2 == 0)):
        raise CorruptStream("words left over")
    return out


# --------------------------------------------------------------------------
# All lanes and segments at once (numpy)
# --------------------------------------------------------------------------

def _layout(n: int, seg_size: int):
    """Segment g holds symbols [g*S, min((g+1)*S, n)); returns (n_seg, steps)."""
    n_seg = max(1, -(-n // seg_size)) if n else 0
    steps = seg_size // LANES if n >= seg_size else -(-n // LANES)
    return n_seg, steps


def encode(sym: np.ndarray, idx: np.ndarray, freq: np.ndarray, cum: np.ndarray,
           seg_size: int) -> list[bytes]:
    """Encode a symbol stream into segments of ``seg_size`` symbols."""
    sym = np.asarray(sym, np.int64)
    idx = np.asarray(idx, np.int64)
    n = sym.size
    if n == 0:
        return []
    assert seg_size % LANES == 0
    n_seg, steps = _layout(n, seg_size)
    gidx = (np.arange(n_seg)[:, None, None] * seg_size
            + np.arange(steps)[None, :, None] * LANES + np.arange(LANES)[None, None, :])
    valid = gidx < n
    g = np.where(valid, gidx, 0)
    f_all = np.where(valid, freq[idx[g], sym[g]], 1).astype(np.uint64)
    c_all = np.where(valid, cum[idx[g], sym[g]], 0).astype(np.uint64)
    x = np.full((n_seg, LANES), L, dtype=np.uint64)
    emit = np.zeros((n_seg, steps, LANES), dtype=bool)
    word = np.zeros((n_seg, steps, LANES), dtype=np.uint64)
    for st in reversed(range(steps)):
        v = valid[:, st, :]
        f = f_all[:, st, :]
        c = c_all[:, st, :]
        e = v & (x >= (f << np.uint64(16)))
        emit[:, st, :] = e
        word[:, st, :] = x & np.uint64(0xFFFF)
        x = np.where(e, x >> np.uint64(16), x)
        q = x // f
        xn = q * np.uint64(M) + (x - q * f) + c
        x = np.where(v, xn, x)
    out = []
    for gi in range(n_seg):
        w = word[gi][emit[gi]].astype(np.uint16)
        if w.size % 2:
            w = np.concatenate([w, np.zeros(1, np.uint16)])
        out.append(x[gi].astype("<u4").tobytes() + w.astype("<u2").tobytes())
    return out


def decode(segments: list[bytes], idx: np.ndarray, freq: np.ndarray, cum: np.ndarray,
           seg_size: int) -> np.ndarray:
    """Decode segments produced by :func:`encode`; raises CorruptStream."""
    idx = np.asarray(idx, np.int64)
    n = idx.size
    n_seg, steps = _layout(n, seg_size)
    if len(segments) != n_seg:
        raise CorruptStream("segment count mismatch")
    if n == 0:
        return np.zeros(0, np.uint8)
    nw = np.zeros(n_seg, np.int64)
    x = np.zeros((n_seg, LANES), np.uint64)
    maxw = 0
    for gi, seg in enumerate(segments):
        if len(seg) < STATE_BYTES or len(seg) % 4:
            raise CorruptStream("segment too short or misaligned")
        nw[gi] = (len(seg) - STATE_BYTES) // 2
        maxw = max(maxw, int(nw[gi]))
    words = np.zeros((n_seg, maxw + LANES), np.uint64)
    for gi, seg in enumerate(segments):
        x[gi] = np.frombuffer(seg[:STATE_BYTES], "<u4").astype(np.uint64)
        words[gi, :nw[gi]] = np.frombuffer(seg[STATE_BYTES:], "<u2").astype(np.uint64)
    gidx = (np.arange(n_seg)[:, None, None] * seg_size
            + np.arange(steps)[None, :, None] * LANES + np.arange(LANES)[None, None, :])
    valid = gidx < n
    kk = idx[np.where(valid, gidx, 0)]
    out = np.zeros((n_seg, steps, LANES), np.uint8)
    pos = np.zeros(n_seg, np.int64)
    freq_u = freq.astype(np.uint64)
    cum_u = cum.astype(np.uint64)
    overrun = np.zeros(n_seg, bool)
    rows = np.arange(n_seg)[:, None]
    for st in range(steps):
        v = valid[:, st, :]
        k = kk[:, st, :]
        slot = x & np.uint64(M - 1)
        s = (cum_u[k] <= slot[..., None]).sum(axis=-1) - 1
        f = freq_u[k, s]
        c = cum_u[k, s]
        xn = f * (x >> np.uint64(PREC)) + slot - c
        need = v & (xn < np.uint64(L))
        rank = np.cumsum(need, axis=1) - need
        rd = pos[:, None] + rank
        overrun |= (need & (rd >= nw[:, None])).any(axis=1)
        w = words[rows, np.minimum(rd, maxw + LANES - 1)]
        xn = np.where(need, (xn << np.uint64(16)) | w, xn)
        x = np.where(v, xn, x)
        out[:, st, :] = np.where(v, s, 0).astype(np.uint8)
        pos += need.sum(axis=1)
    if overrun.any():
        raise CorruptStream("ran out of words")
    if (x != L).any():
        raise CorruptStream("final state is not L")
    for gi in range(n_seg):
        rest = int(nw[gi] - pos[gi])
        if rest == 1 and (words[gi, pos[gi]] == 0 and pos[gi] % 2 == 1):
            continue
        if rest != 0:
            raise CorruptStream("words left over")
    flat = out.reshape(n_seg, steps * LANES)
    res = np.zeros(n, np.uint8)
    for gi in range(n_seg):
        a = gi * seg_size
        b = min(a + seg_size, n)
        res[a:b] = flat[gi, :b - a]
    return res
