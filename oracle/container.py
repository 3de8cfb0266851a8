"""Bit-stream container for one coded chunk (little-endian).

Test infrastructure only (see the package docstring).

  offset  field
   0      u32 magic, the bytes "UFV1"
   4      u16 T, u16 C, u16 H, u16 W        (H, W unpadded)
  12      u8 seg_log2 (y), u8 seg_log2_z (z), u8 k_z, u8 flags
  16      u32 model_tag                     (identifies the weights)
  20      u32 n_seg_z, u32 n_seg_y
  28      u32 seg_bytes[n_seg_z + n_seg_y]
  ...     z segments, then y segments, each a multiple of 4 bytes

flags names the model structure the stream needs (the decoder must run the
same one): bit 0 (FLAG_QUADTREE) = four-step progressive means over the
quadtree partition (Sec. 3.4, Fig. 3 (a)); bit 1 (FLAG_TEMPORAL) = the chunk
is coded conditioned on the temporal context of its stream (Sec. 3.1).
Other bits must be zero.

The paper only says the latent is written to a bit-stream in one interaction
(Sec. 3.4); this layout is this codec's own.  Pins: round trip, and every
malformed-header case raises.
"""
from __future__ import annotations

import struct

MAGIC = b"UFV1"
HEADER = struct.Struct("<4sHHHHBBBBIII")
assert HEADER.size == 28


FLAG_QUADTREE = 1
FLAG_TEMPORAL = 2
KNOWN_FLAGS = FLAG_QUADTREE | FLAG_TEMPORAL


class BadContainer(ValueError):
    pass


def pack(T, C, H, W, seg_log2, seg_log2_z, k_z, model_tag, z_segs, y_segs, flags=0) -> bytes:
    if flags & ~KNOWN_FLAGS:
        raise ValueError("unknown flags")
    hdr = HEADER.pack(MAGIC, T, C, H, W, seg_log2, seg_log2_z, k_z, flags,
                      model_tag & 0xFFFFFFFF, len(z_segs), len(y_segs))
    table = struct.pack(f"<{len(z_segs) + len(y_segs)}I", *[len(s) for s in z_segs + y_segs])
    return hdr + table + b"".join(z_segs) + b"".join(y_segs)


def parse(data: bytes) -> dict:
    if len(data) < HEADER.size:
        raise BadContainer("truncated header")
    (magic, T, C, H, W, sl, slz, kz, flags, tag, nz, ny) = HEADER.unpack_from(data, 0)
    if magic != MAGIC:
        raise BadContainer("bad magic")
    if flags & ~KNOWN_FLAGS:
        raise BadContainer("unknown flags")
    nt = nz + ny
    off = HEADER.size + 4 * nt
    if len(data) < off:
        raise BadContainer("truncated segment table")
    sizes = struct.unpack_from(f"<{nt}I", data, HEADER.size)
    segs = []
    for sz in sizes:
        if sz % 4 or off + sz > len(data):
            raise BadContainer("segment overruns the stream")
        segs.append(data[off:off + sz])
        off += sz
    if off != len(data):
        raise BadContainer("trailing bytes")
    return dict(T=T, C=C, H=H, W=W, seg_log2=sl, seg_log2_z=slz, k_z=kz, flags=flags,
                model_tag=tag, z_segs=segs[:nz], y_segs=segs[nz:])
