"""The tile placement of the tiled step (tile_span in goc_tile.hpp),
compiled from the library's own header as host code and checked
exhaustively on the CPU: every node owned once, tile extents within the
axis, and three nodes of the tile for each one-sided wall difference."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2607_15362_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_tile_span_covers_every_node_and_every_wall_difference():
    tmp = tempfile.mkdtemp()
    try:
        exe = os.path.join(tmp, "tile_span_check")
        subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", CSRC,
                               "-Wno-unused-command-line-argument", "-o", exe,
                               os.path.join(HERE, "host", "tile_span_check.hip")],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
        assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
    finally:
        shutil.rmtree(tmp)
