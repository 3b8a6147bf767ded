"""Host-side logic of the library checked on the CPU (no GPU): the tile run
that the node pass uses to list each band tile a node block covers exactly
once, against brute force over every start, span and axis length up to 70
cells (periodic and not), for each tile size; and the XCD-aware mappings of
workgroups to node blocks, triangle chunks and band-list positions, which
must visit every item exactly once."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2604_17463_amd", "csrc")


def _build(src, out, tmp_path):
    exe = str(tmp_path / out)
    cmd = ["hipcc", "-std=c++17", "-O1", "--offload-host-only", "-I", CSRC, "-o", exe,
           os.path.join(HERE, "host", src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("host build failed:\n" + r.stderr[-2000:])
    return exe


def test_tile_run_lists_each_covered_tile_once(tmp_path):
    exe = _build("tile_run_check.cpp", "tile_run_check", tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "cases ok" in r.stdout


def test_xcd_mappings_visit_every_item_once(tmp_path):
    exe = _build("xcd_map_check.cpp", "xcd_map_check", tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "cases ok" in r.stdout
