// Host-side storage rounding: round-to-nearest-even of a float64 value to
// FP32 / BF16 / FP16 / FP8-E4M3 (OCP, no infinities), saturating at the
// largest finite value, and the bit encodings written to device memory.
//
// Rounding works on the integer significand of the double: drop the bits
// below the target quantum 2^(max(e, emin) - m) with round-half-even on the
// dropped remainder.
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
    switch (dt) {
        case HM_F32: return F32;
        case HM_BF16: return BF16;
        case HM_F16: return F16;
        default: return FP8;
    }
}
}  // namespace

int dtype_bytes(int32_t dt) {
    switch (dt) {
        case HM_F64: return 8;
        case HM_F32: return 4;
        case HM_BF16:
        case HM_F16: return 2;
        case HM_FP8E4M3: return 1;
        default: return 0;
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

}  // namespace hm

extern "C" hm_status hm_round_host(int32_t dtype, const double* in, double* out, int64_t count) {
    if (dtype < HM_F64 || dtype > HM_FP8E4M3 || count < 0 || (count > 0 && (!in || !out))) {
        hm::set_error("hm_round_host: bad dtype or null array");
        return HM_EINVAL;
    }
    for (int64_t i = 0; i < count; ++i) out[i] = hm::round_to(dtype, in[i]);
    return HM_OK;
}
