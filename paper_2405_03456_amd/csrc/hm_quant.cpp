// Host-side storage rounding: round-to-nearest-even of a float64 value to
// FP32 / BF16 / FP16 / FP8-E4M3 (OCP, no infinities) and to the FPX rows of
// Sec. 4.1 (truncated FP32 / FP64 encodings), saturating at the largest
// finite value; the AFLP codec of Sec. 4.1; and the bit encodings written to
// device memory.
//
// Rounding works on the integer significand of the double: drop the bits
// below the target quantum 2^(max(e, emin) - m) with round-half-even on the
// dropped remainder.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "hm_internal.h"

namespace hm {

namespace {
struct Fmt {
    int mant;      // stored mantissa bits
    int emin;      // smallest normal exponent
    int ebits;
    int bias;
    double maxv;
};

const Fmt& fmt(int32_t dt) {
    static const Fmt F32{23, -126, 8, 127, 3.4028234663852886e38};
    static const Fmt BF16{7, -126, 8, 127, 3.3895313892515355e38};
    static const Fmt F16{10, -14, 5, 15, 65504.0};
    static const Fmt FP8{3, -6, 4, 7, 448.0};
    // FPX rows with the FP32 / FP64 exponent: largest finite (2 - 2^-m) 2^emax
    static const Fmt X24{15, -126, 8, 127, std::ldexp(2.0 - std::ldexp(1.0, -15), 127)};
    static const Fmt X40{28, -1022, 11, 1023, std::ldexp(2.0 - std::ldexp(1.0, -28), 1023)};
    static const Fmt X48{36, -1022, 11, 1023, std::ldexp(2.0 - std::ldexp(1.0, -36), 1023)};
    static const Fmt X56{44, -1022, 11, 1023, std::ldexp(2.0 - std::ldexp(1.0, -44), 1023)};
    switch (dt) {
        case HM_F32: return F32;
        case HM_BF16: return BF16;
        case HM_F16: return F16;
        case HM_FPX24: return X24;
        case HM_FPX40: return X40;
        case HM_FPX48: return X48;
        case HM_FPX56: return X56;
        default: return FP8;
    }
}
}  // namespace

bool is_fpx(int32_t dt) { return dt >= HM_FPX24 && dt <= HM_FPX56; }
bool is_aflp(int32_t dt) { return dt >= HM_AFLP8 && dt <= HM_AFLP56; }
int aflp_width(int32_t dt) { return dt - HM_AFLP8 + 1; }
int32_t aflp_dtype(int bytes) { return HM_AFLP8 + bytes - 1; }
bool storage_dtype(int32_t dt) { return (dt >= HM_F64 && dt <= HM_FP8E4M3) || (dt >= HM_FPX24 && dt <= HM_AFLP56); }

int dtype_bytes(int32_t dt) {
    switch (dt) {
        case HM_F64: return 8;
        case HM_F32: return 4;
        case HM_BF16:
        case HM_F16: return 2;
        case HM_FP8E4M3: return 1;
        case HM_FPX24: return 3;
        case HM_FPX40: return 5;
        case HM_FPX48: return 6;
        case HM_FPX56: return 7;
        default: return is_aflp(dt) ? aflp_width(dt) : 0;
    }
}

double dtype_max(int32_t dt) {
    if (dt == HM_F64) return 1.7976931348623157e308;
    return fmt(dt).maxv;
}

double round_to(int32_t dt, double v) {
    if (dt == HM_F64 || v == 0.0 || !std::isfinite(v)) return v;
    const Fmt& f = fmt(dt);
    uint64_t bits;
    std::memcpy(&bits, &v, 8);
    const bool neg = (bits >> 63) != 0;
    int bexp = (int)((bits >> 52) & 0x7FF);
    uint64_t M = bits & ((1ull << 52) - 1);
    int E;                      // exponent of the value's leading bit
    if (bexp == 0) {            // subnormal double: normalise the significand
        int lz = 0;
        while (!(M & (1ull << 52))) {
            M <<= 1;
            ++lz;
        }
        E = -1022 - lz;
    } else {
        M |= (1ull << 52);
        E = bexp - 1023;
    }
    // value = M * 2^(E-52); target quantum exponent
    const int e = E > f.emin ? E : f.emin;
    const int qe = e - f.mant;
    const int shift = qe - (E - 52);
    double r;
    if (shift <= 0) {
        r = std::fabs(v);
    } else {
        uint64_t q, rem, half;
        if (shift >= 63) {
            q = 0;
            rem = M;
            half = 1ull << 62;
        } else {
            q = M >> shift;
            rem = M & ((1ull << shift) - 1);
            half = 1ull << (shift - 1);
        }
        if (rem > half || (rem == half && (q & 1ull))) ++q;
        r = std::ldexp((double)q, qe);
    }
    if (r > f.maxv) r = f.maxv;
    return neg ? -r : r;
}

uint64_t encode(int32_t dt, double v) {
    if (dt == HM_F64) {
        uint64_t b;
        std::memcpy(&b, &v, 8);
        return b;
    }
    if (dt == HM_F32) {
        float x = (float)v;
        uint32_t b;
        std::memcpy(&b, &x, 4);
        return b;
    }
    if (dt == HM_BF16) {
        float x = (float)v;   // exact: v is representable in BF16
        uint32_t b;
        std::memcpy(&b, &x, 4);
        return b >> 16;
    }
    if (is_fpx(dt)) {   // the leading bytes of the FP32 / FP64 encoding
        const int B = dtype_bytes(dt);
        if (dt == HM_FPX24) {
            float x = (float)v;   // exact: v is representable in FPX24
            uint32_t b;
            std::memcpy(&b, &x, 4);
            return b >> 8;
        }
        uint64_t b;
        std::memcpy(&b, &v, 8);
        return b >> (64 - 8 * B);
    }
    const Fmt& f = fmt(dt);
    uint64_t sign = std::signbit(v) ? 1 : 0;
    double a = std::fabs(v);
    uint64_t ef = 0, mf = 0;
    if (a != 0.0) {
        int E = std::ilogb(a);
        if (E < 1 - f.bias) {   // subnormal in the target
            mf = (uint64_t)std::ldexp(a, f.mant - (1 - f.bias));
            ef = 0;
        } else {
            ef = (uint64_t)(E + f.bias);
            mf = (uint64_t)std::ldexp(std::ldexp(a, -E) - 1.0, f.mant);
        }
    }
    const int nbits = 1 + f.ebits + f.mant;
    return (sign << (nbits - 1)) | (ef << f.mant) | mf;
}

// ---------------------------------------------------------------- AFLP
// Codes of Sec. 4.1's AFLP as read here: per column a power-of-two scale
// 2^k with k = floor(log2 vmin) (vmin the smallest nonzero magnitude), so
// every nonzero a = |v| 2^-k >= 1; a = 2^E (1 + f) is stored as z = E + 1 in
// e bits and f rounded to m' = 8B - 1 - e bits; z = 0 is zero.

int m_eps(double eps) {
    // ceil(-log2 eps), exactly: eps = g 2^E with g in [0.5, 1) gives
    // -log2 eps = -E - log2 g, -log2 g in (0, 1]
    int E;
    std::frexp(eps, &E);
    return std::max(0, 1 - E);
}

int aflp_scale_exp(const double* col, int64_t m) {
    double vmin = HUGE_VAL;
    for (int64_t i = 0; i < m; ++i) {
        const double a = std::fabs(col[i]);
        if (a > 0.0 && a < vmin) vmin = a;
    }
    if (vmin == HUGE_VAL) return 0;
    int E;
    std::frexp(vmin, &E);   // vmin = g 2^E, g in [0.5, 1): floor(log2 vmin) = E - 1
    return E - 1;
}

int aflp_column_ebits(const double* col, int64_t m) {
    double vmax = 0.0;
    for (int64_t i = 0; i < m; ++i) vmax = std::max(vmax, std::fabs(col[i]));
    if (vmax == 0.0 || !std::isfinite(vmax)) return 1;   // non-finite data is rejected later
    int E;
    std::frexp(std::ldexp(vmax, -aflp_scale_exp(col, m)), &E);   // largest code z = E
    int bits = 0;
    while ((1 << bits) <= E) ++bits;
    return std::max(1, bits);
}

int aflp_matrix_ebits(const double* A, int64_t m, int64_t k) {
    int e = 1;
    for (int64_t j = 0; j < k; ++j) e = std::max(e, aflp_column_ebits(A + j * m, m));
    return e;
}

bool aflp_feasible(int B, int e) {
    if (B < 1 || B > 7 || 8 * B - 1 - e < 0) return false;
    return e <= (B <= 3 ? 7 : 10);
}

int aflp_direct_width(int e, double eps) {
    int B = std::max(1, (1 + e + m_eps(eps) + 7) / 8);
    while (B <= 7 && !aflp_feasible(B, e)) ++B;
    return B <= 7 ? B : 0;
}

uint64_t aflp_encode(double v, int k, int e, int B, double* value) {
    const int mp = 8 * B - 1 - e;
    const double a = std::ldexp(std::fabs(v), -k);   // exact
    if (a == 0.0) {
        *value = 0.0;
        return 0;
    }
    uint64_t bits;
    std::memcpy(&bits, &a, 8);
    int E = (int)((bits >> 52) & 0x7FF) - 1023;   // a >= 1: a normal double
    const uint64_t sig = (bits & ((1ull << 52) - 1)) | (1ull << 52);
    const int shift = 52 - mp;
    uint64_t q = shift > 0 ? sig >> shift : sig << -shift;   // m' + 1 significant bits
    if (shift > 0) {
        const uint64_t rem = sig & ((1ull << shift) - 1), half = 1ull << (shift - 1);
        if (rem > half || (rem == half && (q & 1ull))) ++q;
    }
    if (q >> (mp + 1)) {   // the carry reached 2^(m'+1): next exponent
        q >>= 1;
        ++E;
    }
    uint64_t z = (uint64_t)(E + 1), M = q & ((1ull << mp) - 1);
    const uint64_t zlim = (1ull << e) - 1;
    if (z > zlim) {   // saturate at the largest code
        z = zlim;
        M = (1ull << mp) - 1;
    }
    const double mag = std::ldexp(1.0 + std::ldexp((double)M, -mp), (int)z - 1 + k);
    const bool neg = std::signbit(v);
    *value = neg ? -mag : mag;
    return ((uint64_t)(neg ? 1 : 0) << (8 * B - 1)) | (z << mp) | M;
}

int32_t fpx_for_eps(double eps) {
    static const int32_t rows[6] = {HM_BF16, HM_FPX24, HM_F32, HM_FPX40, HM_FPX48, HM_FPX56};
    static const int mant[6] = {7, 15, 23, 28, 36, 44};
    const int need = m_eps(eps);
    for (int i = 0; i < 6; ++i)
        if (mant[i] >= need) return rows[i];
    return HM_F64;
}

}  // namespace hm

extern "C" hm_status hm_codec_column(int32_t dtype, double eps, int32_t ebits, const double* col, int64_t m,
                                     double* stored, uint64_t* codes, int32_t* info) {
    using namespace hm;
    if (m < 0 || (m > 0 && (!col || !stored)) || !info) {
        set_error("hm_codec_column: null pointer or negative size");
        return HM_EINVAL;
    }
    for (int64_t i = 0; i < m; ++i)
        if (!std::isfinite(col[i])) {
            set_error("hm_codec_column: non-finite value");
            return HM_EINVAL;
        }
    const bool policy = dtype == HM_AFLP_AUTO || dtype == HM_FPX_AUTO;
    if (!storage_dtype(dtype) && !policy) {
        set_error("hm_codec_column: unsupported dtype");
        return HM_EINVAL;
    }
    if (policy && !(eps > 0.0 && std::isfinite(eps))) {
        set_error("hm_codec_column: a codec policy needs eps > 0");
        return HM_EINVAL;
    }
    int32_t dt = dtype;
    int e = 0;
    if (dtype == HM_AFLP_AUTO || is_aflp(dtype)) {
        e = ebits > 0 ? ebits : aflp_column_ebits(col, m);
        if (dtype == HM_AFLP_AUTO) {
            const int B = aflp_direct_width(e, eps);
            dt = B ? aflp_dtype(B) : HM_F64;
        } else if (!aflp_feasible(aflp_width(dtype), e)) {
            set_error("hm_codec_column: the AFLP width cannot hold this exponent width");
            return HM_EINVAL;
        }
    } else if (dtype == HM_FPX_AUTO) {
        dt = fpx_for_eps(eps);
    }
    info[0] = dt;
    info[1] = dtype_bytes(dt);
    info[2] = is_aflp(dt) ? e : 0;
    info[3] = 0;
    if (is_aflp(dt)) {
        const int k = aflp_scale_exp(col, m);
        info[3] = k;
        for (int64_t i = 0; i < m; ++i) {
            const uint64_t w = aflp_encode(col[i], k, e, aflp_width(dt), stored + i);
            if (codes) codes[i] = w;
        }
        return HM_OK;
    }
    if (dt == HM_F16 || dt == HM_FP8E4M3) {
        set_error("hm_codec_column: column-scaled hardware formats are not codecs (use hm_round_host)");
        return HM_EINVAL;
    }
    for (int64_t i = 0; i < m; ++i) {
        stored[i] = round_to(dt, col[i]);
        if (codes) codes[i] = encode(dt, stored[i]);
    }
    return HM_OK;
}

extern "C" hm_status hm_round_host(int32_t dtype, const double* in, double* out, int64_t count) {
    if (!hm::storage_dtype(dtype) || hm::is_aflp(dtype) || count < 0 || (count > 0 && (!in || !out))) {
        hm::set_error("hm_round_host: bad dtype or null array");
        return HM_EINVAL;
    }
    for (int64_t i = 0; i < count; ++i) out[i] = hm::round_to(dtype, in[i]);
    return HM_OK;
}
