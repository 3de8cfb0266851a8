"""CPU oracle for the chunk codec hot path (test infrastructure, not product).

A plain, slow, obviously correct reimplementation of what the HIP path
computes, in float64 for all real arithmetic and exact Python / uint64
integers for entropy coding.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it; the product library
never does, and this package imports nothing from the product.

Modules
  nets      stand-in transforms: pad, patchify, direct-sum conv, analysis,
            hyper prior, entropy parameters, synthesis, temporal context
            (Sec. 3.1-3.4)
  quadtree  quadtree partition and four-step progressive means (Sec. 3.4,
            Fig. 3 (a))
  entropy   scale table, index thresholds, symbolisation, Gaussian CDF tables
            (Sec. 3.4, the r = round(y - mu) / y = r + mu equations)
  rans      interleaved 32-lane rANS, per segment (arithmetic coder "AE/AD"
            of Fig. 3; the paper does not name its coder)
  container bit-stream layout
  dcblock   the depth-wise convolution block (supplementary DC-block section)
  color     RGB (BT.709) and YUV420 around the YUV444 interface (supplementary
            RGB section)
  codec     encode_chunk / decode_chunk end to end, metrics

Parity status per function is stated in each module header.  The stand-in
network itself has no counterpart in the paper (its trained weights are not
used), so its *behaviour* versus the paper's codec is parity unpinned by
construction; every operation it is built from is pinned.
"""
from . import nets, entropy, rans, container, quadtree, codec, color, dcblock  # noqa: F401
