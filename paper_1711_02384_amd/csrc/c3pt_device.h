// Device helpers of libc3pt: complex arithmetic, MFMA wrappers, small integer
// arithmetic.  gfx950 only.
#pragma once

#include "c3pt_internal.h"

namespace c3pt {

template <typename R>
struct alignas(2 * sizeof(R)) C2 {
    R x, y;
};

template <typename R>
__device__ __forceinline__ C2<R> cadd(C2<R> a, C2<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ C2<R> csub(C2<R> a, C2<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ C2<R> cmul(C2<R> a, C2<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ C2<R> cmulc(C2<R> a, C2<R> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// acc + a * b
template <typename R>
__device__ __forceinline__ C2<R> cfma(C2<R> acc, C2<R> a, C2<R> b) {
    return {acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x};
}
// acc - a * b
template <typename R>
__device__ __forceinline__ C2<R> cfnma(C2<R> acc, C2<R> a, C2<R> b) {
    return {acc.x - a.x * b.x + a.y * b.y, acc.y - a.x * b.y - a.y * b.x};
}
template <typename R>
__device__ __forceinline__ C2<R> cscale(C2<R> a, R s) { return {a.x * s, a.y * s}; }

// Accumulator layouts of the 16x16 MFMAs on gfx950 (lane l, register j):
//   FP32 16x16x4, BF16/FP16 16x16x32: D[4*(l/16) + j][l%16]
//   FP64 16x16x4:                     D[4*j + l/16][l%16]
// kRowsByRegister selects the FP64 form.
template <typename R> struct Mfma;
template <> struct Mfma<float> {
    static constexpr bool kRowsByRegister = false;
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    static constexpr bool kRowsByRegister = true;
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// 16-bit operand types of the split-precision projection.
template <typename T16> struct Mfma16;
template <> struct Mfma16<__bf16> {
    typedef bf16x8 vec_t;
    static __device__ __forceinline__ f32x4 mac(vec_t a, vec_t b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma16<_Float16> {
    typedef f16x8 vec_t;
    static __device__ __forceinline__ f32x4 mac(vec_t a, vec_t b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// v mod L for 0 <= v < 2^20 using a float reciprocal and one correction step.
__device__ __forceinline__ int mod_small(int v, int L, float invL) {
    int q = (int)((float)v * invL);
    int r = v - q * L;
    r += (r < 0) ? L : 0;
    r -= (r >= L) ? L : 0;
    return r;
}

// floor(n / d) for 0 <= n < 2^24, d >= 1, with a float reciprocal and correction.
__device__ __forceinline__ int div_small(int n, int d, float invd) {
    int q = (int)((float)n * invd);
    int r = n - q * d;
    q += (r >= d) ? 1 : 0;
    q -= (r < 0) ? 1 : 0;
    return q;
}

struct TileGeom {
    int V3, L1, L2, L3;
    float inv1, inv12;
    // Tiles that are one segment of an x1 row set row = 1 and give the
    // coordinates of the tile's first site; producers then take neighbour
    // sites from them instead of dividing the site index.
    int row, x1, x2, x3;
};

// Site n -> (x1, x2, x3).
__device__ __forceinline__ void site_xyz(const TileGeom& tg, int n, int& x1, int& x2, int& x3) {
    const int q = div_small(n, tg.L1, tg.inv1);
    x1 = n - q * tg.L1;
    x3 = div_small(n, tg.L1 * tg.L2, tg.inv12);
    x2 = q - x3 * tg.L2;
}

// Coordinates of site t0 + j from those of t0 (x0) by carrying, j >= 0.
__device__ __forceinline__ void site_xyz_from(const TileGeom& tg, const int (&x0)[3], int j, int& x1, int& x2,
                                              int& x3) {
    x1 = x0[0] + j;
    x2 = x0[1];
    x3 = x0[2];
    while (x1 >= tg.L1) {
        x1 -= tg.L1;
        if (++x2 == tg.L2) {
            x2 = 0;
            ++x3;
        }
    }
}

// Neighbour (+- mu, mu = 0, 1, 2, periodic) of the site with coordinates x.
__device__ __forceinline__ int site_shift_xyz(const TileGeom& tg, int x1, int x2, int x3, int mu, int sgn) {
    if (mu == 0) {
        x1 += sgn;
        x1 = (x1 == tg.L1) ? 0 : (x1 < 0 ? tg.L1 - 1 : x1);
    } else if (mu == 1) {
        x2 += sgn;
        x2 = (x2 == tg.L2) ? 0 : (x2 < 0 ? tg.L2 - 1 : x2);
    } else {
        x3 += sgn;
        x3 = (x3 == tg.L3) ? 0 : (x3 < 0 ? tg.L3 - 1 : x3);
    }
    return x1 + tg.L1 * (x2 + tg.L2 * x3);
}

// gamma5 = diag(1, 1, -1, -1) in the DeGrand-Rossi basis: sign of spin s.
template <typename R>
__device__ __forceinline__ R g5(int s) { return s < 2 ? (R)1 : (R)-1; }

}  // namespace c3pt
