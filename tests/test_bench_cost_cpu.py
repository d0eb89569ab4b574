"""Host-only checks of the benchmark's algorithmic byte and flop counts,
the numerators of the roofline figures: each is the per-unit formula of
the kernel table (bytes the launch must move, flops it must do) at the
headline shape, N = 1M items, nnz = 46,020,572 edges, 256 query columns,
r = 1000 (1024 stored), d = 2048."""
import bench

N, NNZ, LDB, RK, B, D = 1_000_000, 46_020_572, 256, 1024, 256, 2048
V = 4.0 * N * LDB  # one fp32 N x ldb vector block


def test_sparse_product_bytes():
    # CSR (int64 row pointers, int32 ids + fp32 values), P gathered once and
    # Q written once (Zs = P in the matrix-core forms)
    by, fl = bench.algorithmic_cost("spmm", N, NNZ, LDB, RK, B, D, 1, 4, True)
    assert by == 8.0 * (N + 1) + 8.0 * NNZ + 2 * V == 2_424_164_584.0
    assert fl == 2.0 * NNZ * LDB
    # fp32 U1 with r > 0 also reads Zs
    by32, _ = bench.algorithmic_cost("spmm", N, NNZ, LDB, RK, B, D, 1, 4, False)
    assert by32 == by + V


def test_similarity_and_combine_bytes_one_pass():
    # bf16 descriptors (2 bytes), queries fp32; the one-pass form writes no
    # B x N score matrix
    two, fl = bench.algorithmic_cost("sim", N, NNZ, LDB, RK, B, D, 1, 2, True, False)
    one, _ = bench.algorithmic_cost("sim", N, NNZ, LDB, RK, B, D, 1, 2, True, True)
    assert two - one == 4.0 * B * N
    assert one == 2.0 * N * D + 4.0 * B * D
    assert fl == 2.0 * B * N * D
    # combine: U1 (two-term bf16: 4 bytes), x read, plus P with the folded
    # last x update
    c1, _ = bench.algorithmic_cost("combine", N, NNZ, LDB, RK, B, D, 1, 4, True, True, False)
    c2, _ = bench.algorithmic_cost("combine", N, NNZ, LDB, RK, B, D, 1, 4, True, True, True)
    assert c1 == 4.0 * N * RK + V
    assert c2 - c1 == V


def test_cg_update_bytes():
    assert bench.algorithmic_cost("update_r", N, NNZ, LDB, RK, B, D, 1)[0] == 3 * V
    assert bench.algorithmic_cost("update_xp", N, NNZ, LDB, RK, B, D, 1)[0] == 5 * V
    # U1 C with the residual update fused: U1, C, and Qs and r read, r written
    by, fl = bench.algorithmic_cost("u_c", N, NNZ, LDB, RK, B, D, 1, 4, True)
    assert by == 4.0 * N * RK + 4.0 * RK * LDB + 3 * V
    assert fl == 2.0 * N * RK * LDB


def test_more_than_one_gpu_is_refused():
    """The benchmark measures one GPU: --gpus N > 1 prints a JSON error line
    and exits 2 before touching a device."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2", "--steps", "1",
                        "--warmup", "0"], capture_output=True, text=True, timeout=120, cwd=root)
    assert p.returncode == 2
    assert "one GPU" in json.loads(p.stdout.strip().splitlines()[-1])["error"]
