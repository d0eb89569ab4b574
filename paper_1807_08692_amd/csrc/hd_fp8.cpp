// FP8 storage form (host side): OCP FP8 E4M3 codes with one fp32 scale per
// column (eigenvectors U1) or per row (descriptors), and the host-only
// quantizer hd_quantize_fp8_e4m3 of the C ABI. The device kernels convert the
// codes to bfloat16 in registers (every E4M3 value is a bfloat16 value) and
// apply the scales to small operands; see k_ugemm_bf16.hip.
#include "hd_internal.h"

#include <cfenv>

namespace hdi {

// OCP FP8 E4M3: sign, 4 exponent bits (bias 7), 3 mantissa bits; exponent
// field 0 holds the subnormals m 2^-9; no infinities; 0x7F / 0xFF are NaN, so
// the largest finite magnitude is 1.75 * 2^8 = 448 (code 0x7E). Rounding is
// to nearest, ties to even; magnitudes at or above 448 saturate to 448.
uint8_t fp8_e4m3_rne(float x) {
    const uint8_t sign = std::signbit(x) ? 0x80 : 0x00;
    const float a = std::fabs(x);
    if (a >= 448.0f) return sign | 0x7E;
    if (a < 0.015625f) {
        // below 2^-6: steps of 2^-9 (a * 512 is exact); q = 8 is the
        // smallest normal value 2^-6, code 0x08, so the code is q itself
        const float q = std::nearbyint(a * 512.0f);
        return sign | (uint8_t)q;
    }
    int e = 0;
    const float f = std::frexp(a, &e);  // a = f 2^e, f in [0.5, 1)
    int E = e - 1;                      // a = (2f) 2^E, 2f in [1, 2)
    float m = std::nearbyint((2.0f * f - 1.0f) * 8.0f);  // exact scaling, then RNE
    if (m == 8.0f) {
        m = 0.0f;
        E += 1;
    }
    if (E > 8 || (E == 8 && m > 6.0f)) return sign | 0x7E;
    return sign | (uint8_t)(((E + 7) << 3) | (int)m);
}

float fp8_e4m3_value(uint8_t b) {
    const int e = (b >> 3) & 15, m = b & 7;
    const float v = e == 0 ? std::ldexp((float)m, -9) : std::ldexp(1.0f + (float)m / 8.0f, e - 7);
    return (b & 0x80) ? -v : v;
}

bool fp8_e4m3_is_nan(uint8_t b) { return (b & 0x7F) == 0x7F; }

void fp8_quantize(int64_t rows, int32_t cols, const float *A, bool per_column, uint8_t *codes, float *scales) {
    // the default rounding mode makes nearbyint round half to even
    const int old = std::fegetround();
    std::fesetround(FE_TONEAREST);
    const int64_t ns = per_column ? cols : rows;
    std::vector<float> mx((size_t)ns, 0.0f);
    for (int64_t i = 0; i < rows; ++i)
        for (int32_t k = 0; k < cols; ++k) {
            const float a = std::fabs(A[(size_t)i * cols + k]);
            float &m = mx[(size_t)(per_column ? k : i)];
            if (a > m) m = a;
        }
    for (int64_t t = 0; t < ns; ++t) scales[t] = mx[(size_t)t] > 0.0f ? mx[(size_t)t] / 448.0f : 1.0f;
    for (int64_t i = 0; i < rows; ++i)
        for (int32_t k = 0; k < cols; ++k) {
            const float s = scales[per_column ? k : i];
            codes[(size_t)i * cols + k] = fp8_e4m3_rne(A[(size_t)i * cols + k] / s);
        }
    std::fesetround(old);
}

}  // namespace hdi

extern "C" int hd_quantize_fp8_e4m3(int64_t rows, int32_t cols, const float *A, int32_t per_column,
                                    uint8_t *codes, float *scales) {
    g_err.clear();
    if (rows < 0 || cols < 0) return fail(HD_EINVAL, "hd_quantize_fp8_e4m3: negative size");
    if (rows == 0 || cols == 0) return HD_OK;
    if (!A || !codes || !scales) return fail(HD_EINVAL, "hd_quantize_fp8_e4m3: NULL array");
    for (int64_t t = 0; t < rows * (int64_t)cols; ++t)
        if (!std::isfinite(A[t])) return fail(HD_EINVAL, "hd_quantize_fp8_e4m3: non-finite input at %lld", (long long)t);
    fp8_quantize(rows, cols, A, per_column != 0, codes, scales);
    return HD_OK;
}
