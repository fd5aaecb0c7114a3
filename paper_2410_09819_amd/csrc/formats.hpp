// Storage classes of a tile (Section IV-C) on the device: rounding from
// binary64, encoding into the class's bits, and decoding back.
//
// Rounding is round-to-nearest-even from binary64 in one step, saturating at
// the class's largest finite value. The quantum of a value x with
// 2^e <= |x| < 2^(e+1) is 2^(max(e, emin) - p + 1) for p significand bits
// and smallest normal exponent emin (which also covers subnormals). Once a
// value is rounded, its conversion to float / half / bfloat16 / e4m3 bits
// is exact.
//
// FP8 is the OCP E4M3 format: 1 sign, 4 exponent bits (bias 7), 3 fraction
// bits, no infinities, largest finite 448, smallest subnormal 2^-9.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc {

enum : int { kFP64 = 0, kFP32 = 1, kFP16 = 2, kBF16 = 3, kFP8 = 4 };

struct FmtSpec {
    int p;        // significand bits
    int emin;     // smallest normal exponent
    double vmax;  // largest finite value
};

__host__ __device__ inline FmtSpec fmt_spec(int c) {
    switch (c) {
        case kFP32: return {24, -126, 3.4028234663852886e38};
        case kFP16: return {11, -14, 65504.0};
        case kBF16: return {8, -126, 3.3895313892515355e38};
        case kFP8: return {4, -6, 448.0};
        default: return {53, -1022, 1.7976931348623157e308};
    }
}

__host__ __device__ inline int fmt_bytes(int c) {
    return c == kFP64 ? 8 : (c == kFP32 ? 4 : (c == kFP8 ? 1 : 2));
}

// Round x (binary64) to class c, result as binary64.
__device__ inline double round_to_class(double x, int c) {
    if (c == kFP64 || x == 0.0 || !(x == x)) return x;
    const FmtSpec f = fmt_spec(c);
    const double ax = fabs(x);
    if (ax >= f.vmax) return x > 0 ? f.vmax : -f.vmax;
    int e = ilogb(ax);
    if (e < f.emin) e = f.emin;
    const int q = e - (f.p - 1);
    double r = rint(ldexp(x, -q));  // exact scaling, RNE to an integer
    r = ldexp(r, q);
    if (fabs(r) > f.vmax) r = x > 0 ? f.vmax : -f.vmax;
    return r;
}

// Encoders of values already representable in the class.
__device__ inline uint16_t enc_fp16(double r) {
    const _Float16 h = (_Float16)(float)r;
    return __builtin_bit_cast(uint16_t, h);
}
__device__ inline uint16_t enc_bf16(double r) {
    return (uint16_t)(__builtin_bit_cast(uint32_t, (float)r) >> 16);
}
__device__ inline uint8_t enc_fp8(double r) {
    uint8_t s = r < 0 ? 0x80 : 0;
    const double a = fabs(r);
    if (a == 0.0) return s;
    const int e = ilogb(a);
    if (e < -6) return s | (uint8_t)(int)ldexp(a, 9);  // subnormal: a = m * 2^-9
    const int m = (int)(ldexp(a, -e) * 8.0) - 8;        // 3 fraction bits
    return s | (uint8_t)((e + 7) << 3) | (uint8_t)m;
}

__device__ inline double dec_fp16(uint16_t b) {
    return (double)(float)__builtin_bit_cast(_Float16, b);
}
__device__ inline double dec_bf16(uint16_t b) {
    return (double)__builtin_bit_cast(float, (uint32_t)b << 16);
}
__device__ inline double dec_fp8(uint8_t b) {
    const int ef = (b >> 3) & 15, m = b & 7;
    const double a = ef == 0 ? ldexp((double)m, -9) : ldexp(1.0 + m * 0.125, ef - 7);
    return (b & 0x80) ? -a : a;
}

// Element i of a tile stored in class c at `base`, times 2^scale.
__device__ inline double load_elem(const void* base, int64_t i, int c, int scale) {
    double v;
    switch (c) {
        case kFP64: return static_cast<const double*>(base)[i];
        case kFP32: v = static_cast<const float*>(base)[i]; break;
        case kFP16: v = dec_fp16(static_cast<const uint16_t*>(base)[i]); break;
        case kBF16: v = dec_bf16(static_cast<const uint16_t*>(base)[i]); break;
        default: v = dec_fp8(static_cast<const uint8_t*>(base)[i]); break;
    }
    return scale ? ldexp(v, scale) : v;
}

// Store binary64 value r (already representable in class c after removing
// 2^scale) as element i of a class-c tile.
__device__ inline void store_elem(void* base, int64_t i, int c, double r) {
    switch (c) {
        case kFP64: static_cast<double*>(base)[i] = r; break;
        case kFP32: static_cast<float*>(base)[i] = (float)r; break;
        case kFP16: static_cast<uint16_t*>(base)[i] = enc_fp16(r); break;
        case kBF16: static_cast<uint16_t*>(base)[i] = enc_bf16(r); break;
        default: static_cast<uint8_t*>(base)[i] = enc_fp8(r); break;
    }
}

// Per-tile power-of-two scale of the narrow-range classes: stored values are
// x * 2^-e with e = ceil(log2(amax / vmax)), which puts the largest entry in
// the top binade. FP64 / FP32 / BF16 tiles are not scaled.
__host__ __device__ inline int class_scale(double amax, int c) {
    if ((c != kFP16 && c != kFP8) || !(amax > 0.0)) return 0;
    const double r = amax / fmt_spec(c).vmax;
    int e = ilogb(r);                  // 2^e <= r < 2^(e+1)
    if (ldexp(1.0, e) < r) e += 1;     // ceil(log2(r))
    return e;
}

}  // namespace tc
