"""The binding works whichever module the caller imports first: a fresh
process that imports the package before torch encodes and decodes a small
chunk, and the decoder reproduces the encoder's stream length."""
import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = """
import sys
sys.path.insert(0, {root!r})
import paper_2606_04410_amd as u   # before torch
import torch
from synthetic import stand_in_weights, video_chunk
c = u.Codec(4, 64, stand_in_weights(4, 64), precision="bf16")
fr = torch.from_numpy(video_chunk(4, 64, 64, 3, seed=1)).cuda()
bs, n = c.encode(fr)
rec = c.decode(bs, n, 64, 64)
c.sync_status()
torch.cuda.synchronize()
assert rec.shape == (4, 3, 64, 64) and n > 28
print("ok", n, flush=True)
c.close()
"""


def test_package_imported_before_torch():
    print("import order: package first, in a fresh process", flush=True)
    r = subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT)], capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1].startswith("ok")
