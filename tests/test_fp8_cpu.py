"""Host-only pins of the FP8 storage form's quantizer (hd_quantize_fp8_e4m3,
no device work): against an independent definition of OCP FP8 E4M3 written
here from its bit layout (sign, four exponent bits with bias 7, three
mantissa bits; exponent field 0 holds the subnormals m 2^-9; 0x7F and 0xFF
are NaN, so 448 is the largest value), rounding to the nearest value with
ties to the even code, and saturation at 448."""
import numpy as np
import pytest

from paper_1807_08692_amd import hd


def e4m3_value(code):
    code = np.asarray(code, np.int64)
    s = np.where(code & 0x80, -1.0, 1.0)
    e = (code >> 3) & 15
    m = code & 7
    v = np.where(e == 0, m * 2.0 ** -9, 2.0 ** (e - 7.0) * (1.0 + m / 8.0))
    return s * v


# the 127 finite non-negative values, ascending with the code
POS = e4m3_value(np.arange(0x7F))


def e4m3_nearest(t):
    """Brute force: the code of the nearest finite value, ties to the even
    code, magnitudes above 448 to 448."""
    t = np.asarray(t, np.float64)
    a = np.minimum(np.abs(t), 448.0)
    d = np.abs(a[:, None] - POS[None, :])
    best = d.min(axis=1, keepdims=True)
    cand = d == best
    # among the nearest (one, or two at a tie) take the even code
    code = np.where(cand[:, ::2].any(axis=1) & (cand.sum(axis=1) > 1),
                    np.argmax(cand & (np.arange(0x7F) % 2 == 0)[None, :], axis=1),
                    np.argmax(cand, axis=1))
    return (code | np.where(np.signbit(t), 0x80, 0)).astype(np.uint8)


def quant(A, per_column):
    return hd.quantize_fp8(np.asarray(A, np.float32), per_column)


def test_value_table_is_the_definition():
    assert POS[0] == 0 and POS[1] == 2.0 ** -9 and POS[8] == 2.0 ** -6 and POS[0x7E] == 448.0
    assert np.all(np.diff(POS) > 0)
    # 2^-9 spacing through the subnormals and the first binade
    assert np.allclose(np.diff(POS[:16]), 2.0 ** -9)


def test_every_code_round_trips():
    # scale 1: one column whose largest magnitude is 448
    vals = e4m3_value(np.arange(0x7F)).astype(np.float32)
    col = np.concatenate([vals, -vals[1:], [448.0]]).astype(np.float32)[:, None]
    codes, sc = quant(col, True)
    assert sc[0] == 1.0
    want = np.concatenate([np.arange(0x7F), 0x80 | np.arange(1, 0x7F), [0x7E]]).astype(np.uint8)
    assert np.array_equal(codes[:, 0], want)


def test_midpoints_round_to_even_and_saturate():
    mids = ((POS[:-1] + POS[1:]) / 2).astype(np.float32)
    assert np.all(mids.astype(np.float64) == (POS[:-1] + POS[1:]) / 2)  # exact in fp32
    col = np.concatenate([mids, [448.0, 455.0, 463.9, 470.0, -1e4]]).astype(np.float32)
    # scale 1 only if the column's largest magnitude is 448: put the big ones
    # in a second column whose scale we check separately
    codes, sc = quant(np.stack([np.concatenate([mids, [448.0] * 5]), col], axis=1), True)
    assert sc[0] == 1.0
    c = codes[: mids.size, 0].astype(np.int64)
    lo = np.arange(mids.size)
    assert np.all((c == lo) | (c == lo + 1))
    assert np.all(c % 2 == 0)  # ties to the even code
    assert np.array_equal(codes[: mids.size, 0], e4m3_nearest(mids))
    # second column: scale = 1e4 / 448 and -1e4 saturates to -448
    assert sc[1] == np.float32(np.float32(1e4) / np.float32(448.0))
    assert codes[-1, 1] == 0x80 | 0x7E


@pytest.mark.parametrize("per_column", [True, False])
def test_random_matrix_against_brute_force(per_column):
    rng = np.random.default_rng(7)
    A = (rng.standard_normal((300, 37)) * np.exp(rng.uniform(-12, 3, size=(300, 37)))).astype(np.float32)
    A[5] = 0.0  # an all-zero row: scale 1 per row
    A[:, 9] = 0.0
    codes, sc = quant(A, per_column)
    mx = np.abs(A).max(axis=0 if per_column else 1)
    want_sc = np.where(mx > 0, (mx.astype(np.float32) / np.float32(448.0)).astype(np.float32), 1.0).astype(np.float32)
    assert np.array_equal(sc, want_sc)
    S = sc[None, :] if per_column else sc[:, None]
    T = (A / S).astype(np.float32)  # the fp32 division of the definition
    want = e4m3_nearest(T.ravel()).reshape(A.shape)
    assert np.array_equal(codes, want)
    # the dequantized matrix is within half a step of A (relative 2^-4 for normals)
    deq = e4m3_value(codes) * S
    rel = np.abs(deq - A) / np.maximum(np.abs(A), 1e-30)
    normal = np.abs(T) >= 2.0 ** -6
    assert np.all(rel[normal] <= 2.0 ** -4 + 1e-7)


def test_rejects_bad_input():
    with pytest.raises(hd.HDError):
        quant(np.array([[1.0, np.nan]], np.float32), True)
    with pytest.raises(hd.HDError):
        quant(np.array([[np.inf]], np.float32), False)
