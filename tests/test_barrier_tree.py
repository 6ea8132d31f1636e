"""The persistent launch's grid-barrier tree, on the CPU: with the blocks
placed on XCDs in any order and number (a census of the hardware XCD IDs
decides the tree, not the block index), every group and XCD of the tree has
exactly one leader per barrier and the global counter reaches the number of
XCDs in use only after the last block arrived.  Built with g++ from the
library's header (paper_1010_2592_amd/csrc/barrier_tree.h)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1010_2592_amd", "csrc")


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("tree") / "barrier_tree_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "barrier_tree_check.cpp"), "-o", exe],
                   check=True)
    return exe


def run(exe, G, xcds, seed):
    text = f"{G} {len(xcds)} {seed}\n" + " ".join(str(int(x)) for x in xcds) + "\n"
    return subprocess.run([exe], input=text, capture_output=True, text=True).stdout.strip()


@pytest.mark.parametrize("seed", range(6))
def test_tree_for_arbitrary_placements(prog, seed):
    rng = np.random.default_rng(seed)
    G = 32
    cases = [
        np.arange(768) % 8,                          # round-robin dispatch, 8 XCDs
        rng.integers(0, 8, 768),                     # any order
        np.sort(rng.integers(0, 8, 517)),            # contiguous ranges, ragged
        rng.integers(0, 3, 200),                     # fewer XCDs in use
        np.full(96, 5),                              # a single XCD
        rng.choice([1, 6], 33),                      # two XCDs, groups of one size
    ]
    for xcds in cases:
        assert run(prog, G, xcds, seed) == "OK"
    assert run(prog, 1, rng.integers(0, 8, 50), seed) == "OK"      # groups of one block
