"""The bench's measurement model (no GPU): the algorithmic bytes per kernel class and the
algorithmic flops of one fast-diagonalisation apply, against the per-unknown figures they are
defined by (each array touched once; complex products counted as four real ones)."""
import dataclasses

import pytest

import bench
import workloads as W


def test_gmres_block_jacobi_bytes_per_unknown():
    N, s, m, bs = 1000, 2, 2, 8  # FP16 storage and inverses, 8-row blocks
    # one working orthogonalisation launch touching 3 basis vectors: w in, v out, inverse row
    # and z out, 3 basis reads
    assert bench.algorithmic_bytes('gm_orth', N, s, m, bs, 1, 3) == N * (2 + 2 + 16 + 2 + 6)
    assert bench.algorithmic_bytes('gm_matvec', N, s, m, bs, 1, 3) == N * (2 + 2 + 6)
    assert bench.algorithmic_bytes('gm_begin', N, s, m, bs, 1, 1) == N * (8 + 2 + 16 + 2)
    assert bench.algorithmic_bytes('residual', N, s, m, bs, 1, 1) == N * 32
    # end of a cycle combining 5 vectors: inverse row, y in and out, 5 basis reads
    assert bench.algorithmic_bytes('gm_finish', N, s, m, bs, 1, 5) == N * (16 + 16 + 10)
    # with the FDM the combination writes t in the arithmetic type instead
    assert bench.algorithmic_bytes('gm_finish', N, s, m, 0, 1, 5, fdm=True, cb=4) == N * (4 + 10)
    # stored directions BJ(v_i): the cycle's end reads no inverse
    assert bench.algorithmic_bytes('gm_finish', N, s, m, bs, 1, 5, zstored=True) == N * (16 + 10)
    # adaptive inverses: FP8 entries (1 byte) in place of the storage type's
    assert bench.algorithmic_bytes('gm_orth', N, s, m, bs, 1, 3, inv_entry=1.0) == N * (2 + 2 + 8 + 2 + 6)
    # work scales with the launches that worked
    assert bench.algorithmic_bytes('residual', N, s, m, bs, 3, 3) == 3 * N * 32


def _prob(n, kind):
    p = W.advdiff_bump(n=8) if kind else W.heat_modes(n=8)
    return dataclasses.replace(p, n=n)


@pytest.mark.parametrize("n", [8, 128, 256])
def test_real_fdm_apply_flops(n):
    # six contractions of 2 n flops per unknown
    assert bench.fdm_apply_flops(_prob(n, 0)) == 6 * 2 * n


@pytest.mark.parametrize("n,H", [(4, 4), (5, 4), (9, 8), (128, 68), (256, 132)])
def test_complex_fdm_apply_flops_on_the_half_spectrum(n, H):
    # x forward real x complex (2 real products, 4 flops per kept frequency), y and z forward and
    # back complex x complex on H of n slices (8 flops per multiply-add), x back real part (4)
    want = 4 * H + 4 * 8 * n * H / n + 4 * H
    assert bench.fdm_apply_flops(_prob(n, 1)) == pytest.approx(want)


def test_complex_fdm_apply_flops_full_spectrum_below_four_points():
    # nx < 4 keeps all frequencies: 40 n, the full-spectrum count
    assert bench.fdm_apply_flops(_prob(3, 1)) == pytest.approx(40 * 3)


def test_csr_spmv_bytes_per_unknown():
    # a CSR SpMV row with 7 nonzeros: values (m) and int32 columns per nonzero, one row pointer,
    # the vector in and out: 7 (m + 4) + 4 + 2 s; FP16 storage -> 50 B, FP64 residual 32 + 88
    N = 1000
    b = bench.algorithmic_bytes('gm_matvec', N, 2, 2, 8, worked=1, units=0, csr_nnz_row=7.0)
    assert b / N == pytest.approx(7 * (2 + 4) + 4 + 2 * 2)
    r = bench.algorithmic_bytes('residual', N, 2, 2, 8, worked=1, units=1, csr_nnz_row=7.0)
    assert r / N == pytest.approx(32 + 7 * 12 + 4)
    # the stencil format moves no matrix
    assert bench.algorithmic_bytes('gm_matvec', N, 2, 2, 8, worked=1, units=0) / N == 4
