"""Host-only check of the fragment order the bfloat16 operands are stored in
(hd::frag_offset, used by the loaders on the host and by the kernels): for
ragged shapes it must map the padded M x K matrix one-to-one onto
[0, M16 K), keep each 16 x 32 tile in one contiguous kilobyte, put the
eight consecutive k of a row in one 16-byte lane piece, and give the 64
lanes of a tile the operand layout of v_mfma_f32_16x16x32_bf16 (lane l:
row l % 16, k from 8 (l / 16)). A small host program built with hipcc
prints every offset; no GPU is used."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1807_08692_amd", "csrc")

PROGRAM = r"""
#include "hd_kernels.h"
#include <cstdio>
#include <cstdlib>
int main(int argc, char **argv) {
    const long M = atol(argv[1]), K = atol(argv[2]);
    for (long m = 0; m < M; ++m)
        for (long k = 0; k < K; ++k) printf("%zu\n", hd::frag_offset(m, k, K / 32));
    return 0;
}
"""


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("frag")
    src = d / "frag.cpp"
    src.write_text(PROGRAM)
    exe = d / "frag"
    p = subprocess.run([hipcc, "-O1", "-std=c++17", "-I" + CSRC, "-x", "hip", "--offload-arch=gfx950",
                        str(src), "-o", str(exe)], capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stderr
    return str(exe)


def offsets(prog, M, K):
    out = subprocess.run([prog, str(M), str(K)], capture_output=True, text=True, timeout=60, check=True)
    return np.array(out.stdout.split(), dtype=np.int64).reshape(M, K)


@pytest.mark.parametrize("M,K", [(16, 32), (37, 64), (48, 96), (5, 160)])
def test_fragment_order(prog, M, K):
    o = offsets(prog, M, K)
    M16 = (M + 15) // 16 * 16
    # one-to-one into the padded matrix's storage
    assert len(np.unique(o)) == M * K
    assert o.min() >= 0 and o.max() < M16 * K
    kt = K // 32
    for mb in range(M16 // 16):
        for kb in range(kt):
            rows = slice(16 * mb, min(16 * mb + 16, M))
            tile = o[rows, 32 * kb:32 * kb + 32]
            base = (mb * kt + kb) * 512
            # the tile is one contiguous kilobyte, tiles in row-major tile order
            assert tile.min() >= base and tile.max() < base + 512
            for r in range(tile.shape[0]):
                for g in range(4):
                    piece = tile[r, 8 * g:8 * g + 8]
                    # eight consecutive k in one 16-byte piece, at lane r + 16 g
                    assert np.array_equal(piece, piece[0] + np.arange(8))
                    assert piece[0] == base + 8 * (r + 16 * g)
