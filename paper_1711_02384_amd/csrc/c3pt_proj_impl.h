// Fused contraction + momentum projection for gfx950 (MI355X): consumers and
// the kernel template, instantiated once per producer in c3pt_proj_*.hip.
//
// One workgroup (4 waves) owns one column block (192 spin-colour components of
// one noise vector / timeslice / operator) and one chunk of spatial sites.
// For every tile of KT sites it
//   1. builds the phases exp(sigma 2 pi i k.(x-r)/L) of the tile from an exact
//      integer phase index into per-direction root-of-unity tables,
//   2. contracts the tile into LDS (the producer, c3pt_producers.h); the
//      global loads for the tile were issued during the previous tile's MFMAs,
//   3. multiplies phases x P on the matrix cores.  The complex product is a
//      real GEMM: the A rows are (re, im) of each momentum, K runs over
//      (site, re/im) of P, and accumulator registers (0,1) / (2,3) of a lane
//      hold (re, im) of two momenta.
// Consumers:
//   NativeCons<float>   FP32 MFMA 16x16x4, FP32 accumulation
//   NativeCons<double>  FP64 MFMA 16x16x4
//   SplitCons<T16>      P and the phases split into hi + lo 16-bit parts
//                       (BF16 or FP16), MFMA 16x16x32 with FP32 accumulation,
//                       three products hi*hi + hi*lo + lo*hi
// FP32 accumulators never span more than kMaxSitesPerChunkF32 sites: each
// workgroup writes its chunk's sums in FP64 and reduce_kernel adds the chunks
// in a fixed order (deterministic, no floating-point atomics).
#pragma once

#include "c3pt_producers.h"

namespace c3pt {

// Phase of momentum m at a site with offsets (d1, d2, d3) = x - r (mod L).
template <typename R>
__device__ __forceinline__ C2<R> phase_at(const PhaseSpec& ph, const C2<R>* tab, int m, int d1, int d2,
                                          int d3, float inv1, float inv2, float inv3) {
    const int i1 = (int)ph.k[0][m] * d1;
    const int i2 = (int)ph.k[1][m] * d2;
    const int i3 = (int)ph.k[2][m] * d3;
    if (ph.cubic) return tab[mod_small(i1 + i2 + i3, ph.L[0], inv1)];
    return cmul(cmul(tab[mod_small(i1, ph.L[0], inv1)], tab[ph.L[0] + mod_small(i2, ph.L[1], inv2)]),
                tab[ph.L[0] + ph.L[1] + mod_small(i3, ph.L[2], inv3)]);
}

// Output rows: lane l, accumulator j of row tile rt hold momentum
// 8*rt + 2*(l/16) + j/2, part j&1 (0 = re, 1 = im), column l%16.
template <typename AccT>
__device__ __forceinline__ void write_tile(const ProjGrid& pg, int chunk, int cb, int rt, int col, int lane,
                                           const AccT& acc) {
    const int n_mom = pg.ph.n_mom;
    const int m0 = 8 * rt + 2 * (lane >> 4);
    const size_t base = ((size_t)chunk * pg.n_colblocks + cb) * (size_t)n_mom;
    if (m0 < n_mom)
        pg.partial[(base + m0) * kBlockCols + col] = make_double2((double)acc[0], (double)acc[1]);
    if (m0 + 1 < n_mom)
        pg.partial[(base + m0 + 1) * kBlockCols + col] = make_double2((double)acc[2], (double)acc[3]);
}

// ---------------------------------------------------------------------------
// Native consumer: FP32 or FP64 MFMA 16x16x4 on P[col][site] (interleaved).
// ---------------------------------------------------------------------------
template <typename R_, int KT_, int MTMAX, int WM, int CT, int MINW_ = 1>
struct NativeCons {
    using R = R_;
    static constexpr int KT = KT_;
    static constexpr int MINW = MINW_;           // minimum waves per SIMD the compiler must allow
    static constexpr int WN = 12 / CT;           // column groups of CT tiles of 16
    static constexpr int NT = 64 * WN * WM;      // WM waves split the row tiles
    static constexpr int RTW = MTMAX / WM;       // row tiles per wave
    static_assert(MTMAX % WM == 0, "row tiles split evenly over waves");
    static constexpr int PST = 2 * KT + 4;       // padded column stride (R elements)
    static constexpr int MROWS = 8 * MTMAX;
    static_assert(WN * CT == 12, "192 columns = 12 tiles of 16");
    using MF = Mfma<R>;
    using acc_t = typename MF::acc_t;
    struct Smem {
        R P[kBlockCols * PST];
        C2<R> ph[KT * MROWS];
    };
    struct Acc {
        acc_t a[RTW][CT];
    };
    struct Sink {
        R* P;
        __device__ __forceinline__ void put(int col, int j, C2<R> v) {
            P[col * PST + 2 * j] = v.x;
            P[col * PST + 2 * j + 1] = v.y;
        }
    };
    static __device__ __forceinline__ Sink sink(Smem& s) { return Sink{s.P}; }
    static __device__ __forceinline__ void zero(Acc& acc) {
#pragma unroll
        for (int i = 0; i < RTW; ++i)
#pragma unroll
            for (int j = 0; j < CT; ++j) acc.a[i][j] = acc_t{0, 0, 0, 0};
    }
    static __device__ __forceinline__ void phases(Smem& s, const C2<R>* tab, const int (*xr)[KT],
                                                  const PhaseSpec& ph, int nsite, int tid, float inv1,
                                                  float inv2, float inv3) {
        for (int e = tid; e < KT * MROWS; e += NT) {
            const int j = e / MROWS, m = e % MROWS;
            C2<R> v = {0, 0};
            if (j < nsite && m < ph.n_mom) v = phase_at(ph, tab, m, xr[0][j], xr[1][j], xr[2][j], inv1, inv2, inv3);
            s.ph[j * MROWS + m] = v;
        }
    }
    static __device__ __forceinline__ void mma(const Smem& s, Acc& acc, int mt, int tid) {
        const int lane = tid & 63, wave = (tid >> 6) % WN, wm = (tid >> 6) / WN;
        // A rows: row r of a tile = (momentum 8*rt + m_off, part); chosen so that the
        // accumulators of both MFMA layouts hold (re, im) pairs in registers (0,1)/(2,3).
        const int arow = lane & 15;
        const int part = MF::kRowsByRegister ? ((arow >> 2) & 1) : (arow & 1);
        const int moff = MF::kRowsByRegister ? (2 * (arow & 3) + (arow >> 3)) : (arow >> 1);
        const int comp = (lane >> 4) & 1;
        const bool take_re = (part == comp);
        const bool negate = (part == 0) && (comp == 1);
        const int asite = lane >> 5;
#pragma unroll 2
        for (int ks = 0; ks < KT / 2; ++ks) {
            R b[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int col = 16 * (wave * CT + ct) + (lane & 15);
                b[ct] = s.P[col * PST + 4 * ks + (lane >> 4)];
            }
#pragma unroll
            for (int rt = 0; rt < RTW; ++rt) {
                const int rtg = wm * RTW + rt;
                if (rtg < mt) {
                    const C2<R> p = s.ph[(2 * ks + asite) * MROWS + 8 * rtg + moff];
                    R av = take_re ? p.x : p.y;
                    av = negate ? -av : av;
#pragma unroll
                    for (int ct = 0; ct < CT; ++ct) acc.a[rt][ct] = MF::mac(av, b[ct], acc.a[rt][ct]);
                }
            }
        }
    }
    static __device__ __forceinline__ void write(const ProjGrid& pg, int chunk, int cb, const Acc& acc, int mt,
                                                 int tid) {
        const int lane = tid & 63, wave = (tid >> 6) % WN, wm = (tid >> 6) / WN;
#pragma unroll
        for (int rt = 0; rt < RTW; ++rt) {
            const int rtg = wm * RTW + rt;
            if (rtg >= mt) continue;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                write_tile(pg, chunk, cb, rtg, 16 * (wave * CT + ct) + (lane & 15), lane, acc.a[rt][ct]);
        }
    }
};

// ---------------------------------------------------------------------------
// Split consumer: P and phases as hi + lo 16-bit values, MFMA 16x16x32.
// K index k = 8*(lane/16) + e of one instruction covers 16 sites: site
// 4*(lane/16) + e/2, component e&1.  KT must be a multiple of 16.
// ---------------------------------------------------------------------------
template <typename T16, int KT_, int MTMAX, int WM, int CT, int MINW_ = 1>
struct SplitCons {
    using R = float;
    static constexpr int KT = KT_;
    static constexpr int MINW = MINW_;
    static constexpr int WN = 12 / CT;
    static constexpr int NT = 64 * WN * WM;
    static constexpr int RTW = MTMAX / WM;
    static_assert(MTMAX % WM == 0, "row tiles split evenly over waves");
    static constexpr int KS = KT / 16;            // MFMA K steps per tile
    static constexpr int PST = 2 * KT + 8;        // padded column stride (16-bit elements)
    static constexpr int MROWS = 8 * MTMAX;
    static_assert(KT % 16 == 0, "split tiles hold whole 16-site K steps");
    static_assert(WN * CT == 12, "192 columns = 12 tiles of 16");
    using MF = Mfma16<T16>;
    using vec_t = typename MF::vec_t;
    struct Smem {
        alignas(16) T16 Phi[kBlockCols * PST];
        alignas(16) T16 Plo[kBlockCols * PST];
        alignas(16) T16 Ahi[KS][MTMAX][64][8];
        alignas(16) T16 Alo[KS][MTMAX][64][8];
    };
    struct Acc {
        f32x4 a[RTW][CT];
    };
    static __device__ __forceinline__ void split(float x, T16& hi, T16& lo) {
        hi = (T16)x;
        lo = (T16)(x - (float)hi);
    }
    struct alignas(4) H2 {
        T16 x, y;
    };
    struct Sink {
        T16* hi;
        T16* lo;
        __device__ __forceinline__ void put(int col, int j, C2<float> v) {
            H2 h, l;
            split(v.x, h.x, l.x);
            split(v.y, h.y, l.y);
            *(H2*)&hi[col * PST + 2 * j] = h;
            *(H2*)&lo[col * PST + 2 * j] = l;
        }
    };
    static __device__ __forceinline__ Sink sink(Smem& s) { return Sink{s.Phi, s.Plo}; }
    static __device__ __forceinline__ void zero(Acc& acc) {
#pragma unroll
        for (int i = 0; i < RTW; ++i)
#pragma unroll
            for (int j = 0; j < CT; ++j) acc.a[i][j] = f32x4{0, 0, 0, 0};
    }
    // A operand of row tile rt, lane 16*g + r, element e: row r = (momentum
    // 8*rt + r/2, part r&1), site 16*ks + 4*g + e/2, component e&1; real row
    // (phi_re, -phi_im), imaginary row (phi_im, phi_re).
    static __device__ __forceinline__ void phases(Smem& s, const C2<float>* tab, const int (*xr)[KT],
                                                  const PhaseSpec& ph, int nsite, int tid, float inv1,
                                                  float inv2, float inv3) {
        for (int e = tid; e < KT * MROWS; e += NT) {
            const int j = e / MROWS, m = e % MROWS;
            C2<float> v = {0, 0};
            if (j < nsite && m < ph.n_mom) v = phase_at(ph, tab, m, xr[0][j], xr[1][j], xr[2][j], inv1, inv2, inv3);
            const int ks = j >> 4, jj = j & 15, g = jj >> 2, e0 = 2 * (jj & 3);
            const int rt = m >> 3, r = 2 * (m & 7);
            T16 h, l;
            split(v.x, h, l);                 // real row, re component; imaginary row, im component
            s.Ahi[ks][rt][16 * g + r][e0] = h;
            s.Alo[ks][rt][16 * g + r][e0] = l;
            s.Ahi[ks][rt][16 * g + r + 1][e0 + 1] = h;
            s.Alo[ks][rt][16 * g + r + 1][e0 + 1] = l;
            split(-v.y, h, l);                // real row, im component
            s.Ahi[ks][rt][16 * g + r][e0 + 1] = h;
            s.Alo[ks][rt][16 * g + r][e0 + 1] = l;
            split(v.y, h, l);                 // imaginary row, re component
            s.Ahi[ks][rt][16 * g + r + 1][e0] = h;
            s.Alo[ks][rt][16 * g + r + 1][e0] = l;
        }
    }
    static __device__ __forceinline__ void mma(const Smem& s, Acc& acc, int mt, int tid) {
        const int lane = tid & 63, wave = (tid >> 6) % WN, wm = (tid >> 6) / WN;
        const int g = lane >> 4;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            vec_t bh[CT], bl[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int col = 16 * (wave * CT + ct) + (lane & 15);
                bh[ct] = *(const vec_t*)&s.Phi[col * PST + 32 * ks + 8 * g];
                bl[ct] = *(const vec_t*)&s.Plo[col * PST + 32 * ks + 8 * g];
            }
#pragma unroll
            for (int rt = 0; rt < RTW; ++rt) {
                const int rtg = wm * RTW + rt;
                if (rtg < mt) {
                    const vec_t ah = *(const vec_t*)&s.Ahi[ks][rtg][lane][0];
                    const vec_t al = *(const vec_t*)&s.Alo[ks][rtg][lane][0];
#pragma unroll
                    for (int ct = 0; ct < CT; ++ct) {
                        acc.a[rt][ct] = MF::mac(al, bh[ct], acc.a[rt][ct]);
                        acc.a[rt][ct] = MF::mac(ah, bl[ct], acc.a[rt][ct]);
                        acc.a[rt][ct] = MF::mac(ah, bh[ct], acc.a[rt][ct]);
                    }
                }
            }
        }
    }
    static __device__ __forceinline__ void write(const ProjGrid& pg, int chunk, int cb, const Acc& acc, int mt,
                                                 int tid) {
        const int lane = tid & 63, wave = (tid >> 6) % WN, wm = (tid >> 6) / WN;
#pragma unroll
        for (int rt = 0; rt < RTW; ++rt) {
            const int rtg = wm * RTW + rt;
            if (rtg >= mt) continue;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                write_tile(pg, chunk, cb, rtg, 16 * (wave * CT + ct) + (lane & 15), lane, acc.a[rt][ct]);
        }
    }
};

// ---------------------------------------------------------------------------
// The fused kernel.
// ---------------------------------------------------------------------------
template <class Cons, template <typename, int, int> class ProdT>
__global__ void __launch_bounds__(Cons::NT, Cons::MINW)
proj_kernel(ProjGrid pg, typename ProdT<typename Cons::R, Cons::KT, Cons::NT>::Args pa) {
    using R = typename Cons::R;
    constexpr int KT = Cons::KT;
    constexpr int NT = Cons::NT;
    using Prod = ProdT<R, KT, NT>;

    __shared__ typename Cons::Smem csm;
    __shared__ typename Prod::Smem psm;
    __shared__ C2<R> sTab[3 * kMaxL];
    __shared__ int sXr[2][3][KT];

    const int tid = threadIdx.x;
    const int cb = blockIdx.x, chunk = blockIdx.y;
    const PhaseSpec& ph = pg.ph;
    const int L1 = ph.L[0], L2 = ph.L[1], L3 = ph.L[2];
    const int mt = (ph.n_mom + 7) >> 3;
    TileGeom tg;
    tg.V3 = pg.V3;
    tg.L1 = L1;
    tg.L2 = L2;
    tg.L3 = L3;
    tg.inv1 = 1.0f / (float)L1;
    tg.inv12 = 1.0f / (float)(L1 * L2);
    const float inv1 = 1.0f / (float)L1, inv2 = 1.0f / (float)L2, inv3 = 1.0f / (float)L3;

    // Root-of-unity tables exp(sigma 2 pi i n / L_j), n < L_j, per direction (FP64 sincospi).
    const int ntab = ph.cubic ? L1 : (L1 + L2 + L3);
    for (int e = tid; e < ntab; e += NT) {
        int n = e, Lj = L1;
        if (e >= L1) {
            if (e >= L1 + L2) { n = e - L1 - L2; Lj = L3; }
            else { n = e - L1; Lj = L2; }
        }
        double sn, cs;
        sincospi(2.0 * (double)n / (double)Lj, &sn, &cs);
        sTab[e] = {(R)cs, (R)(ph.sigma * sn)};
    }

    auto coords = [&](int t0, int buf) {
        if (tid < KT) {
            int x0[3], x1, x2, x3;
            site_xyz(tg, t0, x0[0], x0[1], x0[2]);
            site_xyz_from(tg, x0, tid, x1, x2, x3);
            int d1 = x1 - ph.r[0], d2 = x2 - ph.r[1], d3 = x3 - ph.r[2];
            sXr[buf][0][tid] = d1 + ((d1 < 0) ? L1 : 0);
            sXr[buf][1][tid] = d2 + ((d2 < 0) ? L2 : 0);
            sXr[buf][2][tid] = d3 + ((d3 < 0) ? L3 : 0);
        }
    };

    typename Cons::Acc acc;
    Cons::zero(acc);
    const int s_lo = chunk * pg.chunk_sites;
    const int s_hi = min(pg.V3, s_lo + pg.chunk_sites);
    typename Prod::Regs rg;
    if (s_lo < s_hi) {
        Prod::load(pa, tg, cb, s_lo, min(KT, s_hi - s_lo), rg, tid);
        coords(s_lo, 0);
    }
    __syncthreads();
    int buf = 0;
    for (int t0 = s_lo; t0 < s_hi; t0 += KT) {
        const int nsite = min(KT, s_hi - t0);
        Cons::phases(csm, sTab, sXr[buf], ph, nsite, tid, inv1, inv2, inv3);
        auto sink = Cons::sink(csm);
        Prod::store(pa, tg, cb, t0, nsite, rg, psm, sink, tid);
        const int t1 = t0 + KT;
        if (t1 < s_hi) {
            Prod::load(pa, tg, cb, t1, min(KT, s_hi - t1), rg, tid);
            coords(t1, buf ^ 1);
        }
        __syncthreads();
        Cons::mma(csm, acc, mt, tid);
        __syncthreads();
        buf ^= 1;
    }
    Cons::write(pg, chunk, cb, acc, mt, tid);
}

// ---------------------------------------------------------------------------
// Variants: (site tile KT, row split WM) per momentum-tile class; index 0 is
// the default, others are picked by the autotuner (c3pt_set_variant).
// ---------------------------------------------------------------------------
template <class Cons, template <typename, int, int> class ProdT>
hipError_t launch_cons(const ProjGrid& pg, const typename ProdT<float, 16, 256>::Args& a, hipStream_t st) {
    dim3 grid(pg.n_colblocks, pg.n_chunks);
    hipLaunchKernelGGL((proj_kernel<Cons, ProdT>), grid, dim3(Cons::NT), 0, st, pg, a);
    return hipGetLastError();
}

template <template <typename, int, int> class ProdT, template <typename, int, int, int, int> class Cons,
          typename T>
hipError_t launch_variant(int mt, int variant, const ProjGrid& pg, const typename ProdT<float, 16, 256>::Args& a,
                          hipStream_t st) {
    if (mt <= 4) {
        if (variant == 0) return launch_cons<Cons<T, 16, 4, 1, 3>, ProdT>(pg, a, st);
        if (variant == 1) return launch_cons<Cons<T, 32, 4, 1, 3>, ProdT>(pg, a, st);
    } else if (mt <= 8) {
        if (variant == 0) return launch_cons<Cons<T, 16, 8, 2, 3>, ProdT>(pg, a, st);
        if (variant == 1) return launch_cons<Cons<T, 32, 8, 2, 3>, ProdT>(pg, a, st);
        if (variant == 2) return launch_cons<Cons<T, 16, 8, 1, 3>, ProdT>(pg, a, st);
    } else if (mt <= 12) {
        if (variant == 0) return launch_cons<Cons<T, 16, 12, 2, 3>, ProdT>(pg, a, st);
        if (variant == 1) return launch_cons<Cons<T, 32, 12, 2, 3>, ProdT>(pg, a, st);
        if (variant == 2) return launch_cons<Cons<T, 16, 12, 1, 3>, ProdT>(pg, a, st);
    } else if (mt <= 16) {
        if (variant == 0) return launch_cons<Cons<T, 16, 16, 2, 3>, ProdT>(pg, a, st);
        if (variant == 1) return launch_cons<Cons<T, 32, 16, 2, 3>, ProdT>(pg, a, st);
    }
    return hipErrorInvalidValue;
}

template <typename T, int KT, int MTMAX, int WM, int CT>
using NativeConsT = NativeCons<T, KT, MTMAX, WM, CT>;

template <template <typename, int, int> class ProdT>
hipError_t dispatch(int mode, int mt, int variant, const ProjGrid& pg,
                    const typename ProdT<float, 16, 256>::Args& a, hipStream_t st) {
    switch (mode) {
        case kModeF64:
            if (mt <= 4 && variant == 0) return launch_cons<NativeCons<double, 16, 4, 1, 3>, ProdT>(pg, a, st);
            return hipErrorInvalidValue;
        case kModeF32:
            return launch_variant<ProdT, NativeConsT, float>(mt, variant, pg, a, st);
        case kModeSplitBF16:
            return launch_variant<ProdT, SplitCons, __bf16>(mt, variant, pg, a, st);
        case kModeSplitF16:
            return launch_variant<ProdT, SplitCons, _Float16>(mt, variant, pg, a, st);
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace c3pt
