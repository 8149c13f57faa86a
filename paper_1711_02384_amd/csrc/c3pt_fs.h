// Fused contraction + factored projection on split 16-bit MFMA (gfx950).
//
// The contracted tensors of Eqs. (9)-(10) all have the form
//   P(x)[at][X] = sum_c u(x)[at][c] B(x)[c][X]
// with a short colour sum c (3 terms), an "A index" at (4 values: the
// insertion's antiquark spin, or the spectator's noise spin b') and 48
// "B columns" X:
//   insertion, Eq. (10):   u = g[at] conj(s[(at,c)]),          B[c][(bt,b,c0)] = G[(bt,c)][(b,c0)]
//   meson spectator, (9):  u = g[b'] eta[(b',c)],               B[c][(a',a,c0)] = g[a'] g[a] conj(G[(a',c)][(a,c0)])
//   nucleon spectator:     u = g[b'] eta[(b',c)],               B[c][(q,c')]    = Q[q][c][c'] (the diquark)
//   derivatives, Eq. (10): u = the transported noise (see below), B = G.
// The first stage of the factored projection (the sum over x1 with
// w1^(k1 x1)) is a GEMM over K = (c, x1, re/im), so the colour contraction
// is folded into it:
//   R1[k1][at][X] = sum_{x1, c} (w1^(k1 x1) u(x)[at][c]) B(x)[c][X].
// A = w1^(k1 x1) u is formed per tile in FP32 and split into hi + lo 16-bit
// parts; B is split the same way, either when its tile is staged or once per
// call by a pass before the launch (fs_split_kernel; the nucleon's diquark is
// always formed and split by its pass, fs_diquark_kernel).  Three MFMA 16x16x32 products
// hi*hi + hi*lo + lo*hi accumulate in FP32 (the error per product is about
// 2^-22 relative for FP16, 2^-16 for BF16).  Stages 2 and 3 (over x2 and x3)
// are the FP32 register and partial-sum updates of the factored kernel.
//
// Derivative operators: the derivative of Eq. (10) acts on G at y +- nu.
// Shifting the summation site moves it onto the noise side, so every
// operator reads the same B = G(y') of one timeslice:
//   sum_y phi(y) t+(y) G(y+nu) = e^{-i sigma p_nu} sum_y' phi(y') t+(y'-nu) G(y'),
//   sum_y phi(y) t-(y) G(y-nu) = e^{+i sigma p_nu} sum_y' phi(y') t-(y'+nu) G(y'),
// with t+(y) = 1/2 v(y) U_nu(y), t-(y) = 1/2 v(y) U_nu(y-nu)^dag, v = g conj(s)
// (for nu = t the two parts read G on tau+1 and tau-1 at the same site).
// Each (nu, +-) is its own column block ("slot") of partial sums; the FP64
// reduction applies the per-momentum factors and forms the difference.
//
// Workgroup: 4 CB waves = CB column blocks (noise vectors of one slot,
// sharing the B tile in LDS; CB = 1, 2 or 3) x four A indices; a wave owns
// one A index and all 48 B columns as three 16-column MFMA tiles.  Three
// blocks give twelve waves (three per SIMD) and share the propagator tile's
// split three ways.  The tile loop is the factored kernel's: tiles are KT
// sites of one x1 row, one workgroup barrier per tile, B and u of the next
// tile staged while the current one is computed; within a tile the A
// operands of the next K step are formed while the MFMAs of the current one
// issue.
#pragma once

#include "c3pt_device.h"
#include "c3pt_fs_api.h"

#include <utility>

namespace c3pt {

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// One group of four consecutive sites of one B plane in the split form:
// hi parts (re, im) of the four sites, then the lo parts.
struct alignas(16) FsGroup {
    uint4 hi, lo;
};

template <typename T16>
__device__ __forceinline__ void fs_split(float x, T16& hi, T16& lo) {
    hi = (T16)x;
    lo = (T16)(x - (float)hi);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
template <typename T16>
struct FsHalf2 {
    typedef T16 type __attribute__((ext_vector_type(2)));
};

// Split of two FP32 values into packed hi and lo 16-bit pairs.  The
// residuals v - hi are exact in FP32; for FP16 each is one mixed-precision
// FMA that reads its half of the packed hi directly (v_fma_mix_f32:
// -hi * 1 + v), instead of a conversion back to FP32 and a subtraction.
template <typename T16>
__device__ __forceinline__ void fs_split2(f32x2 v, unsigned& hi, unsigned& lo) {
    using h2 = typename FsHalf2<T16>::type;
    const h2 h = __builtin_convertvector(v, h2);
    __builtin_memcpy(&hi, &h, 4);
    f32x2 r;
    if constexpr (__is_same(T16, _Float16)) {
        float r0, r1;
        asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r0) : "v"(hi), "v"(v.x));
        asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r1) : "v"(hi), "v"(v.y));
        r = f32x2{r0, r1};
    } else {
        r = v - __builtin_convertvector(h, f32x2);
    }
    const h2 l = __builtin_convertvector(r, h2);
    __builtin_memcpy(&lo, &l, 4);
}

template <typename T16>
__device__ __forceinline__ unsigned fs_pack(T16 a, T16 b) {
    unsigned short ua, ub;
    __builtin_memcpy(&ua, &a, 2);
    __builtin_memcpy(&ub, &b, 2);
    return (unsigned)ua | ((unsigned)ub << 16);
}

// f(integral_constant<int, I>) for I = 0 .. N-1, expanded at compile time
// (register arrays indexed by I stay in registers whatever the unroller does).
template <class F, int... I>
__device__ __forceinline__ void fs_expand(F& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void fs_unroll(F&& f) {
    fs_expand(f, std::make_integer_sequence<int, N>{});
}

template <int KT, int CB>
struct FsShape {
    static constexpr int NT = 256 * CB;            // threads: CB column blocks x four A indices
    static constexpr int GB = KT / 4;              // four-site groups per tile
    static constexpr int PSTR = GB * 32 + 16;      // LDS bytes per B plane (padded against bank conflicts)
    static constexpr int HS = KT / 16;             // MFMA K steps per summed colour (16 sites x re/im)
    static constexpr int W1S = KT + 2;             // W1 row stride (complex), padded (fs_dyn_bytes)
    static constexpr int NB16 = kFsPlanes * GB * 2;          // 16-byte pieces of a B tile
    static constexpr int KB = (NB16 + NT - 1) / NT;
    static_assert(KB * NT <= 2 * NB16, "repeated B pieces stay within the tile");
    static constexpr int NG = kFsPlanes * GB;      // four-site groups of a tile (FP32 source)
    static constexpr int KG = (NG + NT - 1) / NT;
    static_assert(KG * NT <= 2 * NG, "repeated groups stay within the tile");
    static constexpr int NU = 12 * CB * KT;        // staged u values per tile (CB blocks x 12 x KT)
    static constexpr int KU = (NU + NT - 1) / NT;
};

template <int KT, int CB>
struct FsSmem {
    using S = FsShape<KT, CB>;
    alignas(16) unsigned char B[2][kFsPlanes * S::PSTR];
    alignas(16) C2<float> U[2][CB][12][KT];                  // [buffer][block][3 at + c][x1]
    C2<float> coef2[2][kFacMaxPairsF32 + kFacMaxBPerA];
    FactorPlan plan;
};
// The lattice-sized tables follow in dynamic LDS (fs_dyn_bytes): W1
// [nseg][kFacMaxK1][W1S], w1^(k1 (seg KT + x1)), zero for unused slots and
// sites past the row; then the root tables w_j^x for x < L_j, j = 1, 2, 3.

template <typename T16, int KT, int KIND, bool BSPLIT, int CB>
__global__ void __launch_bounds__(256 * CB) fs_kernel(ProjGrid pg, FsArgs fa) {
    using S = FsShape<KT, CB>;
    constexpr int NT = S::NT;
    using MF = Mfma16<T16>;
    using vec_t = typename MF::vec_t;
    __shared__ FsSmem<KT, CB> sm;
    extern __shared__ __attribute__((aligned(16))) float2 fs_dyn[];
    const int tid = threadIdx.x;
    const int lane = tid & 63, g = lane >> 4, cl = lane & 15;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int cbj = wave >> 2, at = wave & 3;
    // work item (within, share, chunk), chunk outermost; consecutive items run
    // on one XCD (one share and chunk read the same slice; neighbouring
    // shares read each other's as the time derivative's neighbours)
    const int nw = gridDim.x, w = blockIdx.x;
    const int full = (nw / 8) * 8;
    const int item = (w < full) ? (w % 8) * (nw / 8) + w / 8 : w;
    const int within = item % pg.n_per_share;
    const int rest = item / pg.n_per_share;
    const int share = rest % pg.n_share;
    const int chunk = rest / pg.n_share;
    const int N = fa.N;
    const int ngroup = (N + CB - 1) / CB;
    const int slot = within / ngroup;
    const int i0 = CB * (within % ngroup);
    const bool valid = i0 + cbj < N;   // an odd noise count leaves the second block of the last pair empty
    const int cb = (((fa.i_base + min(i0 + cbj, N - 1)) * fa.n_share + share) * fa.n_slots + slot);
    const int L1 = fa.L[0], L2 = fa.L[1], L3 = fa.L[2];
    const int V3 = L1 * L2 * L3;
    const float inv1 = 1.0f / (float)L1, inv2 = 1.0f / (float)L2, inv3 = 1.0f / (float)L3;
    const int nseg = (L1 + KT - 1) / KT;
    C2<float>* const W1 = (C2<float>*)fs_dyn;                        // [nseg][kFacMaxK1][W1S]
    C2<float>* const root0 = W1 + nseg * kFacMaxK1 * S::W1S;         // [L1], then [L2], [L3]
    C2<float>* const root1 = root0 + L1;
    C2<float>* const root2 = root1 + L2;
    // B source of this work item: a split block, or the FP32 propagator slice
    // of the slot (tau_j, tau_j + 1 for (t, +), tau_j - 1 for (t, -))
    const int role = KIND == 2 && slot == 7 ? 1 : (KIND == 2 && slot == 8 ? 2 : 0);
    const unsigned char* Bg =
        (const unsigned char*)fa.B + (size_t)(KIND == 0 ? slot : fa.bidx[share][role]) * fa.b_stride;
    const C2<float>* Gsrc = (const C2<float>*)fa.G[KIND == 0 ? 0 : share][role];
    // derivative slot: direction and sign
    const int nu = slot >= 1 ? (slot - 1) >> 1 : -1;
    const int sgn = slot >= 1 ? (slot - 1) & 1 : 0;
    const C2<float>* ubase = (const C2<float>*)fa.u0[KIND == 0 ? 0 : share];
    const C2<float>* Ulink = KIND == 2 ? (const C2<float>*)(nu == 3 && sgn == 1 ? fa.Up[share] : fa.U[share]) : nullptr;

    // ---- setup: plan, root tables, w1 of every row segment -------------
    {
        const int* src = (const int*)pg.phase;
        int* dst = (int*)&sm.plan;
        for (int i = tid; i < (int)(sizeof(FactorPlan) / sizeof(int)); i += NT) dst[i] = src[i];
        const int sigma = ((const FactorPlan*)pg.phase)->sigma;
        for (int i = tid; i < L1 + L2 + L3; i += NT) {
            const int j = i < L1 ? 0 : (i < L1 + L2 ? 1 : 2);
            const int x = i - (j == 0 ? 0 : (j == 1 ? L1 : L1 + L2));
            const int L = fa.L[j];
            double sn, cs;
            sincospi(2.0 * (double)x / (double)L, &sn, &cs);
            root0[i] = C2<float>{(float)cs, (float)(sigma * sn)};
        }
    }
    __syncthreads();
    for (int e = tid; e < nseg * kFacMaxK1 * KT; e += NT) {
        const int seg = e / (kFacMaxK1 * KT), rem = e % (kFacMaxK1 * KT);
        const int a = rem / KT, x = rem % KT;
        const int x1 = seg * KT + x;
        C2<float> wv = {0.f, 0.f};
        if (a < sm.plan.n1 && x1 < L1) wv = root0[mod_small(sm.plan.k1[a] * x1, L1, inv1)];
        W1[(seg * kFacMaxK1 + a) * S::W1S + x] = wv;
    }
    const int n_mom = sm.plan.n_mom, n12 = sm.plan.n12;
    // stage-2 ownership: k1 slots 2g, 2g+1 of the lane's three columns; nbmax
    // (uniform) bounds the stage-2 updates of every lane
    int nbmax = 0;
    for (int a = 0; a < sm.plan.n1; ++a) nbmax = max(nbmax, sm.plan.bstart[a + 1] - sm.plan.bstart[a]);
    nbmax = __builtin_amdgcn_readfirstlane(nbmax);
    int bs[2], nb[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int a = 2 * g + h;
        bs[h] = a < sm.plan.n1 ? sm.plan.bstart[a] : 0;
        nb[h] = a < sm.plan.n1 ? sm.plan.bstart[a + 1] - bs[h] : 0;
    }
    int colX[3];
#pragma unroll
    for (int ct = 0; ct < 3; ++ct) {
        const int X = 16 * ct + cl;
        colX[ct] = fa.colmap == 0 ? at * 48 + X : (X / 3) * 12 + at * 3 + X % 3;
    }

    const int p0 = chunk * pg.chunk_planes;
    const int p1 = min(L3, p0 + pg.chunk_planes);
    const int n_tiles = (p1 - p0) * L2 * nseg;

    struct TilePos {
        int seg, x2, x3, row;
    };
    auto advance = [&](TilePos q) __attribute__((always_inline)) {
        if (++q.seg == nseg) {
            q.seg = 0;
            ++q.row;
            if (++q.x2 == L2) {
                q.x2 = 0;
                ++q.x3;
            }
        }
        return q;
    };

    // ---- staging of one tile: B pieces and the u values of both blocks --
    u32x4 breg[BSPLIT ? S::KB : 1];
    C2<float> greg[BSPLIT ? 1 : S::KG][4];
    // FP32 source: plane offset and first site of each of the thread's groups
    // (groups past the tile's end repeat earlier ones: the same value is stored twice)
    unsigned goff[BSPLIT ? 1 : S::KG];
    int gi4[BSPLIT ? 1 : S::KG];
    if constexpr (!BSPLIT) {
        fs_unroll<S::KG>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            const int e0 = tid + k * NT;
            const int e = e0 < S::NG ? e0 : e0 - S::NG;
            const int p = e / S::GB, X = p % 48, cs = p / 48;
            goff[k] = (unsigned)((3 * (X / 12) + cs) * 12 + X % 12) * (unsigned)V3;
            gi4[k] = 4 * (e % S::GB);
        });
    }
    C2<float> sreg[S::KU][KIND == 2 ? 3 : 1];
    C2<float> lreg[S::KU][KIND == 2 ? 3 : 1];
    auto load_tile = [&](const TilePos& q) __attribute__((always_inline)) {
        // split blocks are [row][plane][Lp / 4] groups: the tile's 144 plane
        // segments lie within one row's span
        const size_t rowoff = (size_t)(q.x2 + L2 * q.x3) * kFsPlanes * (size_t)(fa.Lp / 4) + (size_t)q.seg * S::GB;
        if constexpr (BSPLIT) {
            fs_unroll<S::KB>([&](auto kc) __attribute__((always_inline)) {
                constexpr int k = decltype(kc)::value;
                // pieces past the tile's end repeat earlier ones (the same value is
                // stored twice), so every thread loads and stores unconditionally
                const int e0 = tid + k * NT;
                const int e = e0 < S::NB16 ? e0 : e0 - S::NB16;
                const int p = e / (2 * S::GB), r = e % (2 * S::GB);
                breg[k] = *(const u32x4*)(Bg + ((size_t)p * (size_t)(fa.Lp / 4) + rowoff) * 32 + r * 16);
            });
        } else {
            const unsigned rowL1 = (unsigned)(L1 * (q.x2 + L2 * q.x3));
            const int segKT = q.seg * KT;
            fs_unroll<S::KG>([&](auto kc) __attribute__((always_inline)) {
                constexpr int k = decltype(kc)::value;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    greg[k][j] = Gsrc[goff[k] + rowL1 + (unsigned)min(segKT + gi4[k] + j, L1 - 1)];
            });
        }
        fs_unroll<S::KU>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            // threads past the last entry repeat it (same load, same value stored)
            const int e = min(tid + k * NT, S::NU - 1);
            const int bj = e / (12 * KT), rem = e % (12 * KT);
            const int A = rem / KT, xl = rem % KT;
            const int x1 = min(q.seg * KT + xl, L1 - 1);
            const int noise = fa.i_base + min(i0 + bj, N - 1);
            const C2<float>* src = ubase + (size_t)noise * 12 * V3;
            const int n = x1 + L1 * (q.x2 + L2 * q.x3);
            if (KIND != 2 || slot == 0) {
                sreg[k][0] = src[(size_t)A * V3 + n];
            } else {
                const int atk = A / 3, d = A % 3;
                // site of s and of the link
                int xs[3] = {x1, q.x2, q.x3};
                int xu[3] = {x1, q.x2, q.x3};
                if (nu < 3) {
                    const int Ln = fa.L[nu];
                    const int xm = xs[nu] == 0 ? Ln - 1 : xs[nu] - 1;
                    const int xp = xs[nu] == Ln - 1 ? 0 : xs[nu] + 1;
                    if (sgn == 0) {
                        xs[nu] = xm;
                        xu[nu] = xm;
                    } else {
                        xs[nu] = xp;
                    }
                }
                const int ns = xs[0] + L1 * (xs[1] + L2 * xs[2]);
                const int nl = xu[0] + L1 * (xu[1] + L2 * xu[2]);
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    sreg[k][cc] = src[(size_t)(3 * atk + cc) * V3 + ns];
                    // + : U_nu[c][d] ; - : U_nu[d][c] (conjugated below)
                    const int e9 = sgn == 0 ? cc * 3 + d : d * 3 + cc;
                    lreg[k][cc] = Ulink[(size_t)((nu * 9) + e9) * V3 + nl];
                }
            }
        });
    };
    auto store_tile = [&](const TilePos& q, int buf) __attribute__((always_inline)) {
        if constexpr (BSPLIT) {
            fs_unroll<S::KB>([&](auto kc) __attribute__((always_inline)) {
                constexpr int k = decltype(kc)::value;
                const int e0 = tid + k * NT;
                const int e = e0 < S::NB16 ? e0 : e0 - S::NB16;
                const int p = e / (2 * S::GB), r = e % (2 * S::GB);
                *(u32x4*)(sm.B[buf] + p * S::PSTR + r * 16) = breg[k];
            });
        } else {
            fs_unroll<S::KG>([&](auto kc) __attribute__((always_inline)) {
                constexpr int k = decltype(kc)::value;
                const int e0 = tid + k * NT;
                const int e = e0 < S::NG ? e0 : e0 - S::NG;
                const int p = e / S::GB, gi = e % S::GB;
                const int X = p % 48;
                // Sites past the row's end hold copies of its last site (finite):
                // their A entries are zero (W1 and u vanish there), so they add nothing.
                u32x4 hi, lo;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    f32x2 v = {greg[k][j].x, greg[k][j].y};
                    if constexpr (KIND == 0) {
                        // meson spectator (the only in-kernel split of KIND 0): g[a'] g[a] conj(G)
                        const float sg = (X / 12 < 2 ? 1.f : -1.f) * ((X % 12) / 3 < 2 ? 1.f : -1.f);
                        v = f32x2{sg * v.x, -sg * v.y};
                    }
                    unsigned h, l;
                    fs_split2<T16>(v, h, l);
                    hi[j] = h;
                    lo[j] = l;
                }
                unsigned char* dst = sm.B[buf] + p * S::PSTR + gi * 32;
                *(u32x4*)dst = hi;
                *(u32x4*)(dst + 16) = lo;
            });
        }
        fs_unroll<S::KU>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            // threads past the last entry repeat it (same load, same value stored)
            const int e = min(tid + k * NT, S::NU - 1);
            const int bj = e / (12 * KT), rem = e % (12 * KT);
            const int A = rem / KT, xl = rem % KT;
            const int atk = A / 3;
            const bool inrow = q.seg * KT + xl < L1;
            const float sg = atk < 2 ? 1.f : -1.f;
            C2<float> u;
            if (KIND == 0) {
                u = {sg * sreg[k][0].x, sg * sreg[k][0].y};                 // g eta
            } else if (KIND == 1 || slot == 0) {
                u = {sg * sreg[k][0].x, -sg * sreg[k][0].y};                // g conj(s)
            } else {
                u = {0.f, 0.f};
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    const C2<float> v = {sg * sreg[k][cc].x, -sg * sreg[k][cc].y};
                    u = sgn == 0 ? cfma(u, v, lreg[k][cc]) : cadd(u, cmulc(v, lreg[k][cc]));
                }
                u = cscale(u, 0.5f);
            }
            sm.U[buf][bj][A][xl] = inrow ? u : C2<float>{0.f, 0.f};
        });
    };
    auto fill_coef2 = [&](int par, int x2) __attribute__((always_inline)) {
        for (int b = tid; b < n12 + kFacMaxBPerA; b += NT)
            sm.coef2[par][b] = b < n12 ? root1[mod_small(sm.plan.k2[b] * x2, L2, inv2)] : C2<float>{0.f, 0.f};
    };

    f32x4 acc[3];
    // pairs per k1 slot held in registers: fewer with three column blocks per
    // workgroup (the host plans those launches with at most kFsPairsCB3)
    constexpr int NBP = CB == 3 ? kFsPairsCB3 : kFacMaxBPerA;
    C2<float> r2[3][2][NBP];
#pragma unroll
    for (int ct = 0; ct < 3; ++ct) {
        acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int i = 0; i < NBP; ++i) r2[ct][h][i] = C2<float>{0.f, 0.f};
    }
    if (n_tiles <= 0) return;   // uniform: no barrier follows

    // pa: the tile computed, pb: the next (staged during it), pc: the one after
    // (loaded during it); past the end pb and pc repeat the last tile
    TilePos pa = {0, 0, p0, 0};
    TilePos pb = n_tiles > 1 ? advance(pa) : pa;
    TilePos pc = n_tiles > 2 ? advance(pb) : pb;
    load_tile(pa);
    __syncthreads();            // W1 and the plan are in LDS
    store_tile(pa, 0);
    fill_coef2(0, pa.x2);
    if (n_tiles > 1) load_tile(pb);
    __syncthreads();

    const int a_row = cl >> 1, part = cl & 1;
    for (int T = 0; T < n_tiles; ++T) {
        const int par = T & 1;
        const int seg = pa.seg, x3 = pa.x3, row = pa.row;
        const bool row_end = (seg == nseg - 1);
        const bool plane_end = row_end && pa.x2 == L2 - 1;
        // ---- stage 1: A = w1 u (split), B from LDS, three products ----
        // row (a, part) of the real form: part 0 takes (Re z, -Im z), part 1
        // (Im z, Re z) of z = w u; as linear maps of (u.x, u.y):
        //   v0 = c0 u.x + c1 u.y,  v1 = c1 u.x - c0 u.y
        // (one 16-site half: with longer tiles each step reads its own, which
        // keeps the registers of one half live instead of all)
        auto make_cf = [&](int h, float (&c)[4][2]) __attribute__((always_inline)) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const C2<float> wv = W1[(seg * kFacMaxK1 + a_row) * S::W1S + 16 * h + 4 * g + j];
                c[j][0] = part ? wv.y : wv.x;
                c[j][1] = part ? wv.x : -wv.y;
            }
        };
        float cf1[4][2];
        if constexpr (S::HS == 1) make_cf(0, cf1);
        // Steps st = (cs, h) in order, each nine MFMAs (three column tiles ct x
        // three products).  The A operands of step st + 1 are formed (VALU)
        // while the MFMAs of step st issue, and the B operands of each column
        // tile are read from LDS one tile ahead.
        auto form_a = [&](int st, vec_t& ahi, vec_t& alo) __attribute__((always_inline)) {
            const int cs = st / S::HS, h = st % S::HS;
            float cfs[4][2];
            if constexpr (S::HS > 1) make_cf(h, cfs);
            const float(&cf)[4][2] = S::HS == 1 ? cf1 : cfs;
            u32x4 ah, al;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const C2<float> uv = sm.U[par][cbj][3 * at + cs][16 * h + 4 * g + j];
                const f32x2 v = {cf[j][0] * uv.x + cf[j][1] * uv.y, cf[j][1] * uv.x - cf[j][0] * uv.y};
                unsigned hh, ll;
                fs_split2<T16>(v, hh, ll);
                ah[j] = hh;
                al[j] = ll;
            }
            ahi = __builtin_bit_cast(vec_t, ah);
            alo = __builtin_bit_cast(vec_t, al);
        };
        auto read_b = [&](int sub, vec_t& bhi, vec_t& blo) __attribute__((always_inline)) {
            const int st = sub / 3, ct = sub % 3;
            const int cs = st / S::HS, h = st % S::HS;
            const unsigned char* bp = sm.B[par] + (48 * cs + 16 * ct + cl) * S::PSTR + (4 * h + g) * 32;
            bhi = *(const vec_t*)bp;
            blo = *(const vec_t*)(bp + 16);
        };
        constexpr int NST = 3 * S::HS;
        // The insertion on 32-site tiles has no registers to spare for the
        // overlap: it forms and reads each step's operands in place and stages
        // the next tiles after the MFMAs.
        constexpr bool kPipe = !(KIND == 2 && KT == 32);
        vec_t a_hi[2], a_lo[2], b_hi[2], b_lo[2];
        if constexpr (kPipe) {
            read_b(0, b_hi[0], b_lo[0]);
            form_a(0, a_hi[0], a_lo[0]);
        }
        // The steps run at raised wave priority, stage 2 and the tile barrier
        // at the normal one: the SIMD's arbiter then favours waves still in
        // their MFMA steps over waves already past them (measured: insertion
        // 2.80 -> 2.72 ms, spectator 2.55 -> 2.50 ms at 48^3; raising it
        // from the start of the tile, or through stage 2, gained less).
        __builtin_amdgcn_s_setprio(1);
        fs_unroll<3 * NST>([&](auto subc) __attribute__((always_inline)) {
            constexpr int sub = decltype(subc)::value;
            constexpr int st = sub / 3, ct = sub % 3;
            constexpr int ca = kPipe ? st & 1 : 0, cb2 = kPipe ? sub & 1 : 0;
            if constexpr (!kPipe) {
                if constexpr (ct == 0) form_a(st, a_hi[0], a_lo[0]);
                read_b(sub, b_hi[0], b_lo[0]);
            } else {
                if constexpr (sub + 1 < 3 * NST) read_b(sub + 1, b_hi[cb2 ^ 1], b_lo[cb2 ^ 1]);
                if constexpr (ct == 0 && st + 1 < NST) form_a(st + 1, a_hi[ca ^ 1], a_lo[ca ^ 1]);
                if constexpr (ct == 0 && st + 1 == NST) {
                    // the last step's MFMAs run beside the staging of the next
                    // tile (into the other buffer, last read before the previous
                    // barrier) and the loads of the one after; past the end both
                    // repeat the last tile, which nothing reads again
                    store_tile(pb, par ^ 1);
                    load_tile(pc);
                }
            }
            acc[ct] = MF::mac(a_lo[ca], b_hi[cb2], acc[ct]);
            acc[ct] = MF::mac(a_hi[ca], b_lo[cb2], acc[ct]);
            acc[ct] = MF::mac(a_hi[ca], b_hi[cb2], acc[ct]);
            if constexpr (kPipe && ct == 2) {
                // interleave the step's MFMAs with the next step's A formation,
                // or with the staging after the last step (three VALU per MFMA:
                // 13.60 -> 13.49 ms per 48^3 step against four; two or six
                // were no better than four)
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, st);   // one MFMA
                    __builtin_amdgcn_sched_group_barrier(0x002, 3, st);   // three VALU
                }
            }
        });
        __builtin_amdgcn_s_setprio(0);
        if (row_end) {
            // ---- stage 2: over x2, in registers -------------------------
            // coefficients of the lane's pairs, read together (the table is
            // zero-padded by kFacMaxBPerA entries)
            const C2<float>* cf = sm.coef2[row & 1];
            C2<float> cw[2][NBP];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int i = 0; i < NBP; ++i) cw[h][i] = cf[bs[h] + i];
#pragma unroll
            for (int i = 0; i < NBP; ++i) {
                if (i >= nbmax) break;   // uniform
#pragma unroll
                for (int h = 0; h < 2; ++h) {
#pragma unroll
                    for (int ct = 0; ct < 3; ++ct) {
                        const C2<float> v =
                            h == 0 ? C2<float>{acc[ct][0], acc[ct][1]} : C2<float>{acc[ct][2], acc[ct][3]};
                        r2[ct][h][i] = cfma(r2[ct][h][i], cw[h][i], v);
                    }
                }
            }
#pragma unroll
            for (int ct = 0; ct < 3; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (plane_end) {
                // ---- stage 3: over x3, into the chunk's partial sums ----
                float2* part_out = (float2*)pg.partial;
                const size_t base = ((size_t)chunk * pg.n_colblocks + cb) * (size_t)n_mom;
                const bool first = (x3 == p0);
#pragma unroll
                for (int ct = 0; ct < 3; ++ct) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
#pragma unroll
                        for (int i = 0; i < NBP; ++i) {
                            if (i < nb[h]) {
                                const int b = bs[h] + i;
                                for (int jm = sm.plan.mstart[b]; jm < sm.plan.mstart[b + 1]; ++jm) {
                                    const int m = sm.plan.m_of[jm];
                                    const C2<float> w3 = root2[mod_small(sm.plan.k3[m] * x3, L3, inv3)];
                                    C2<float> v = cmul(w3, r2[ct][h][i]);
                                    if (valid) {
                                        float2& dst = part_out[(base + m) * kBlockCols + colX[ct]];
                                        if (!first) {
                                            const float2 o = dst;
                                            v.x += o.x;
                                            v.y += o.y;
                                        }
                                        dst = float2{v.x, v.y};
                                    }
                                }
                            }
                            r2[ct][h][i] = C2<float>{0.f, 0.f};
                        }
                    }
                }
            }
        }
        if constexpr (!kPipe) {
            store_tile(pb, par ^ 1);
            load_tile(pc);
        }
        // ---- the next tile's stage-2 coefficients (the other row parity)
        if (T + 1 < n_tiles && pb.seg == 0) fill_coef2(pb.row & 1, pb.x2);
        __syncthreads();
        pa = pb;
        pb = pc;
        if (T + 3 < n_tiles) pc = advance(pc);
    }
}

}  // namespace c3pt
