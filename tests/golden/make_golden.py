"""Writes the golden fixtures of this folder from the CPU oracle alone.

c1_bitstream.sha256: SHA-256 of the bit-stream the oracle produces for the
small configuration (T=4 RGB frames of 64x64, C=64, generator seed 1, max
shift 3, seg_log2 = 14, seg_log2_z = 10, model tag 0x55F00401).  It freezes the
container and coder format: any change to either changes this hash.

Run:  python tests/golden/make_golden.py
"""
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import codec  # noqa: E402
from synthetic import stand_in_weights, video_chunk  # noqa: E402


def main():
    fr = video_chunk(4, 64, 64, 3, seed=1)
    w = stand_in_weights(4, 64)
    bs, _ = codec.encode_chunk(fr, w, seg_log2=14, seg_log2_z=10, model_tag=0x55F00401)
    with open(os.path.join(HERE, "c1_bitstream.sha256"), "w") as f:
        f.write(hashlib.sha256(bs).hexdigest() + "  c1 (T=4, 64x64, C=64, seed 1)\n")
    with open(os.path.join(HERE, "c1_bitstream.bin"), "wb") as f:
        f.write(bs)


if __name__ == "__main__":
    main()
