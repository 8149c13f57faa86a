// Fused contraction + momentum projection for gfx950 (MI355X): consumers and
// the kernel template, instantiated once per producer in c3pt_proj_*.hip.
//
// One workgroup owns one column block (192 spin-colour components of one
// noise vector / timeslice / operator) and one chunk of spatial sites.  For
// every tile of KT sites it
//   1. copies the tile's phases from the phase table (c3pt_phase.hip) into LDS,
//   2. contracts the tile into LDS (the producer, c3pt_producers.h),
//   3. multiplies phases x P on the matrix cores.  The complex product is a
//      real GEMM: the A rows are (re, im) of each momentum, K runs over
//      (site, re/im) of P, and accumulator registers (0,1) / (2,3) of a lane
//      hold (re, im) of two momenta.
// The global loads of tile t+1 (inputs and phases) are issued before the
// MFMA loop of tile t.
// Consumers:
//   NativeCons<float>   FP32 MFMA 16x16x4, FP32 accumulation
//   NativeCons<double>  FP64 MFMA 16x16x4
//   SplitCons<T16>      P and the phases split into hi + lo 16-bit parts
//                       (BF16 or FP16), MFMA 16x16x32 with FP32 accumulation,
//                       three products hi*hi + hi*lo + lo*hi
// FP32 accumulators never span more than kMaxSitesPerChunkF32 sites: each
// workgroup stores its chunk's sums in the accumulator type and the reduction
// adds the chunks in FP64 in a fixed order (deterministic, no floating-point
// atomics).  Phases are taken at the origin; the reduction applies the source
// offset as a per-momentum factor.
#pragma once

#include "c3pt_producers.h"

namespace c3pt {

// Partial sums are stored in the accumulator's own type (complex float or
// complex double): storing them loses nothing.
template <typename E> struct PartialT;
template <> struct PartialT<float> { typedef float2 type; };
template <> struct PartialT<double> { typedef double2 type; };

// Output rows: lane l, accumulator j of row tile rt hold momentum
// 8*rt + 2*(l/16) + j/2, part j&1 (0 = re, 1 = im), column l%16.
template <typename E, typename AccT>
__device__ __forceinline__ void write_tile(void* partial, int n_colblocks, int n_mom, int chunk, int cb, int rt,
                                           int col, int lane, const AccT& acc) {
    using P2 = typename PartialT<E>::type;
    P2* part = (P2*)partial;
    const int m0 = 8 * rt + 2 * (lane >> 4);
    const size_t base = ((size_t)chunk * n_colblocks + cb) * (size_t)n_mom;
    if (m0 < n_mom) part[(base + m0) * kBlockCols + col] = P2{acc[0], acc[1]};
    if (m0 + 1 < n_mom) part[(base + m0 + 1) * kBlockCols + col] = P2{acc[2], acc[3]};
}

// Copy of one tile of the phase table (TB bytes, contiguous) through registers.
template <int TB, int NT>
struct TableTile {
    static constexpr int kN = (TB / 16 + NT - 1) / NT;
    struct Regs {
        float4 v[kN];
    };
    static __device__ __forceinline__ void load(const char* src, Regs& r, int tid) {
        const float4* s4 = (const float4*)src;
#pragma unroll
        for (int i = 0; i < kN; ++i) {
            const int idx = tid + i * NT;
            if (idx < TB / 16) r.v[i] = s4[idx];
        }
    }
    static __device__ __forceinline__ void store(char* dst, const Regs& r, int tid) {
        float4* d4 = (float4*)dst;
#pragma unroll
        for (int i = 0; i < kN; ++i) {
            const int idx = tid + i * NT;
            if (idx < TB / 16) d4[idx] = r.v[i];
        }
    }
};

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
    static constexpr int PST = 2 * KT + 4;       // padded column stride (R elements)
    static constexpr int MROWS = 8 * MTMAX;
    static constexpr int TB = KT * MROWS * (int)sizeof(C2<R>);   // phase bytes per tile
    static_assert(MTMAX % WM == 0, "row tiles split evenly over waves");
    static_assert(WN * CT == 12, "192 columns = 12 tiles of 16");
    using MF = Mfma<R>;
    using acc_t = typename MF::acc_t;
    using Tab = TableTile<TB, NT>;
    struct Smem {
        R P[kBlockCols * PST];
        alignas(16) C2<R> ph[KT * MROWS];
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
    static __device__ __forceinline__ const char* table_tile(const void* tab, int t0) {
        return (const char*)tab + (size_t)t0 * MROWS * sizeof(C2<R>);
    }
    static __device__ __forceinline__ char* lds_table(Smem& s) { return (char*)s.ph; }
    static __device__ __forceinline__ void zero(Acc& acc) {
#pragma unroll
        for (int i = 0; i < RTW; ++i)
#pragma unroll
            for (int j = 0; j < CT; ++j) acc.a[i][j] = acc_t{0, 0, 0, 0};
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
    static __device__ __forceinline__ void write(void* partial, int n_colblocks, int n_mom, int chunk, int cb,
                                                 const Acc& acc, int mt, int tid) {
        const int lane = tid & 63, wave = (tid >> 6) % WN, wm = (tid >> 6) / WN;
#pragma unroll
        for (int rt = 0; rt < RTW; ++rt) {
            const int rtg = wm * RTW + rt;
            if (rtg >= mt) continue;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                write_tile<R>(partial, n_colblocks, n_mom, chunk, cb, rtg, 16 * (wave * CT + ct) + (lane & 15), lane,
                              acc.a[rt][ct]);
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
    static constexpr int KS = KT / 16;            // MFMA K steps per tile
    static constexpr int PST = 2 * KT + 8;        // padded column stride (16-bit elements)
    static constexpr int TB = KS * 2 * MTMAX * 64 * 8 * 2;   // phase bytes per tile
    static_assert(MTMAX % WM == 0, "row tiles split evenly over waves");
    static_assert(KT % 16 == 0, "split tiles hold whole 16-site K steps");
    static_assert(WN * CT == 12, "192 columns = 12 tiles of 16");
    using MF = Mfma16<T16>;
    using vec_t = typename MF::vec_t;
    using Tab = TableTile<TB, NT>;
    struct Smem {
        alignas(16) T16 Phi[kBlockCols * PST];
        alignas(16) T16 Plo[kBlockCols * PST];
        alignas(16) T16 A[KS][2][MTMAX][64][8];   // [k step][hi, lo][row tile][lane][e]
    };
    struct Acc {
        f32x4 a[RTW][CT];
    };
    struct alignas(4) H2 {
        T16 x, y;
    };
    static __device__ __forceinline__ void split(float x, T16& hi, T16& lo) {
        hi = (T16)x;
        lo = (T16)(x - (float)hi);
    }
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
    static __device__ __forceinline__ const char* table_tile(const void* tab, int t0) {
        return (const char*)tab + (size_t)(t0 / 16) * (2 * MTMAX * 64 * 8 * 2);
    }
    static __device__ __forceinline__ char* lds_table(Smem& s) { return (char*)&s.A[0][0][0][0][0]; }
    static __device__ __forceinline__ void zero(Acc& acc) {
#pragma unroll
        for (int i = 0; i < RTW; ++i)
#pragma unroll
            for (int j = 0; j < CT; ++j) acc.a[i][j] = f32x4{0, 0, 0, 0};
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
                    const vec_t ah = *(const vec_t*)&s.A[ks][0][rtg][lane][0];
                    const vec_t al = *(const vec_t*)&s.A[ks][1][rtg][lane][0];
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
    static __device__ __forceinline__ void write(void* partial, int n_colblocks, int n_mom, int chunk, int cb,
                                                 const Acc& acc, int mt, int tid) {
        const int lane = tid & 63, wave = (tid >> 6) % WN, wm = (tid >> 6) / WN;
#pragma unroll
        for (int rt = 0; rt < RTW; ++rt) {
            const int rtg = wm * RTW + rt;
            if (rtg >= mt) continue;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                write_tile<float>(partial, n_colblocks, n_mom, chunk, cb, rtg, 16 * (wave * CT + ct) + (lane & 15), lane,
                              acc.a[rt][ct]);
        }
    }
};

// ---------------------------------------------------------------------------
// Tile loop over sites [s_lo, s_hi) of one column block.
// ---------------------------------------------------------------------------
template <class Cons, class Prod>
__device__ __forceinline__ void tile_loop(const typename Prod::Ctx& ctx, const TileGeom& tg, const void* phase,
                                          int s_lo, int s_hi, typename Cons::Smem& csm, typename Prod::Smem& psm,
                                          typename Cons::Acc& acc, int mt, int tid) {
    constexpr int KT = Cons::KT;
    using Tab = typename Cons::Tab;
    typename Prod::Regs rg;
    typename Tab::Regs tr;
    if (s_lo < s_hi) {
        Prod::load(ctx, tg, s_lo, min(KT, s_hi - s_lo), rg, tid);
        Tab::load(Cons::table_tile(phase, s_lo), tr, tid);
    }
    for (int t0 = s_lo; t0 < s_hi; t0 += KT) {
        const int nsite = min(KT, s_hi - t0);
        Tab::store(Cons::lds_table(csm), tr, tid);
        auto sink = Cons::sink(csm);
        Prod::store(ctx, tg, t0, nsite, rg, psm, sink, tid);
        const int t1 = t0 + KT;
        if (t1 < s_hi) {
            Prod::load(ctx, tg, t1, min(KT, s_hi - t1), rg, tid);
            Tab::load(Cons::table_tile(phase, t1), tr, tid);
        }
        __syncthreads();
        Cons::mma(csm, acc, mt, tid);
        __syncthreads();
    }
}

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

    const int tid = threadIdx.x;
    // Work item; consecutive items (same shared input slice and chunk) go to the
    // same XCD: workgroup w runs on XCD w % 8.
    const int nw = gridDim.x, w = blockIdx.x;
    const int full = (nw / 8) * 8;
    const int item = (w < full) ? (w % 8) * (nw / 8) + w / 8 : w;
    const int within = item % pg.n_per_share;
    const int rest = item / pg.n_per_share;
    const int share = rest % pg.n_share;
    const int chunk = rest / pg.n_share;
    const int cb = Prod::colblock(pa, share, within);
    const typename Prod::Ctx ctx = Prod::resolve(pa, pg.V3, cb);
    const int mt = (pg.n_mom + 7) >> 3;
    TileGeom tg;
    tg.V3 = pg.V3;
    tg.L1 = pa.L[0];
    tg.L2 = pa.L[1];
    tg.L3 = pa.L[2];
    tg.inv1 = 1.0f / (float)tg.L1;
    tg.inv12 = 1.0f / (float)(tg.L1 * tg.L2);
    tg.row = tg.x1 = tg.x2 = tg.x3 = 0;

    typename Cons::Acc acc;
    Cons::zero(acc);
    const int s_lo = chunk * pg.chunk_sites;
    const int s_hi = min(pg.V3, s_lo + pg.chunk_sites);
    tile_loop<Cons, Prod>(ctx, tg, pg.phase, s_lo, s_hi, csm, psm, acc, mt, tid);
    Cons::write(pg.partial, pg.n_colblocks, pg.n_mom, chunk, cb, acc, mt, tid);
}

// ---------------------------------------------------------------------------
// Persistent form for batches: every workgroup takes (job, column block,
// chunk) items from a queue until it is empty.  The queue head is a plain
// integer counter (no floating-point atomics; each item is summed by exactly
// one workgroup, so the result does not depend on the schedule).
// ---------------------------------------------------------------------------
template <class Cons, template <typename, int, int> class ProdT>
__global__ void __launch_bounds__(Cons::NT, Cons::MINW) batch_kernel(BatchGrid bg) {
    using R = typename Cons::R;
    constexpr int KT = Cons::KT;
    constexpr int NT = Cons::NT;
    using Prod = ProdT<R, KT, NT>;

    __shared__ typename Cons::Smem csm;
    __shared__ typename Prod::Smem psm;
    __shared__ int s_item;

    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(bg.counter, 1);
        __syncthreads();
        // the item is the same for the whole workgroup: make that visible to the
        // compiler so that everything derived from it stays in scalar registers
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (it >= bg.n_items) break;
        const int4 item = bg.items[it];
        const BatchJob& job = bg.jobs[item.x];
        const int cb = item.y, chunk = item.z;
        const typename Prod::Ctx ctx = Prod::resolve(job, job.V3, cb);
        TileGeom tg;
        tg.V3 = job.V3;
        tg.L1 = job.L[0];
        tg.L2 = job.L[1];
        tg.L3 = job.L[2];
        tg.inv1 = 1.0f / (float)tg.L1;
        tg.inv12 = 1.0f / (float)(tg.L1 * tg.L2);
    tg.row = tg.x1 = tg.x2 = tg.x3 = 0;
        typename Cons::Acc acc;
        Cons::zero(acc);
        const int s_lo = chunk * job.chunk_sites;
        const int s_hi = min(job.V3, s_lo + job.chunk_sites);
        const int mt = (job.n_mom + 7) >> 3;
        tile_loop<Cons, Prod>(ctx, tg, job.phase, s_lo, s_hi, csm, psm, acc, mt, tid);
        Cons::write(job.partial, job.n_colblocks, job.n_mom, chunk, cb, acc, mt, tid);
    }
}

// ---------------------------------------------------------------------------
// Variants: (site tile KT, row split WM) per momentum-tile class; index 0 is
// the default, others are picked by the autotuner (c3pt_set_variant).
// ---------------------------------------------------------------------------
template <class Cons, template <typename, int, int> class ProdT>
hipError_t launch_cons(const ProjGrid& pg, const typename ProdT<float, 16, 256>::Args& a, hipStream_t st) {
    dim3 grid(pg.n_colblocks * pg.n_chunks);
    hipLaunchKernelGGL((proj_kernel<Cons, ProdT>), grid, dim3(Cons::NT), 0, st, pg, a);
    return hipGetLastError();
}

template <template <typename, int, int> class ProdT, template <typename, int, int, int, int, int> class Cons,
          typename T>
hipError_t launch_variant(int mt, int variant, const ProjGrid& pg, const typename ProdT<float, 16, 256>::Args& a,
                          hipStream_t st) {
    if (mt <= 4) {
        if (variant == 0) return launch_cons<Cons<T, 16, 4, 1, 3, 1>, ProdT>(pg, a, st);
        if (variant == 1) return launch_cons<Cons<T, 32, 4, 1, 3, 1>, ProdT>(pg, a, st);
    } else if (mt <= 8) {
        if (variant == 0) return launch_cons<Cons<T, 16, 8, 2, 3, 1>, ProdT>(pg, a, st);
        if (variant == 1) return launch_cons<Cons<T, 32, 8, 2, 3, 1>, ProdT>(pg, a, st);
        if (variant == 2) return launch_cons<Cons<T, 16, 8, 1, 3, 1>, ProdT>(pg, a, st);
    } else if (mt <= 12) {
        if (variant == 0) return launch_cons<Cons<T, 16, 12, 2, 3, 1>, ProdT>(pg, a, st);
        if (variant == 1) return launch_cons<Cons<T, 32, 12, 2, 3, 1>, ProdT>(pg, a, st);
        if (variant == 2) return launch_cons<Cons<T, 16, 12, 1, 3, 1>, ProdT>(pg, a, st);
    } else if (mt <= 16) {
        if (variant == 0) return launch_cons<Cons<T, 16, 16, 2, 3, 1>, ProdT>(pg, a, st);
        if (variant == 1) return launch_cons<Cons<T, 32, 16, 2, 3, 1>, ProdT>(pg, a, st);
    }
    return hipErrorInvalidValue;
}

template <class Cons, template <typename, int, int> class ProdT>
hipError_t launch_batch_cons(const BatchGrid& bg, int n_wg, hipStream_t st) {
    hipLaunchKernelGGL((batch_kernel<Cons, ProdT>), dim3(n_wg), dim3(Cons::NT), 0, st, bg);
    return hipGetLastError();
}

template <class Cons, template <typename, int, int> class ProdT>
int batch_occupancy() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<Cons, ProdT>, Cons::NT, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

// Split / FP32 batch variants mirror launch_variant.
template <template <typename, int, int> class ProdT, template <typename, int, int, int, int, int> class Cons,
          typename T>
int batch_variant(int mt, int variant, const BatchGrid* bg, int n_wg, hipStream_t st, hipError_t* err) {
#define C3PT_BV(KT_, MT_, WM_)                                                          \
    {                                                                                   \
        using C = Cons<T, KT_, MT_, WM_, 3, 1>;                                         \
        if (bg) *err = launch_batch_cons<C, ProdT>(*bg, n_wg, st);                      \
        return batch_occupancy<C, ProdT>();                                             \
    }
    if (mt <= 4) {
        if (variant == 0) C3PT_BV(16, 4, 1)
        if (variant == 1) C3PT_BV(32, 4, 1)
    } else if (mt <= 8) {
        if (variant == 0) C3PT_BV(16, 8, 2)
        if (variant == 1) C3PT_BV(32, 8, 2)
        if (variant == 2) C3PT_BV(16, 8, 1)
    } else if (mt <= 12) {
        if (variant == 0) C3PT_BV(16, 12, 2)
        if (variant == 1) C3PT_BV(32, 12, 2)
        if (variant == 2) C3PT_BV(16, 12, 1)
    } else if (mt <= 16) {
        if (variant == 0) C3PT_BV(16, 16, 2)
        if (variant == 1) C3PT_BV(32, 16, 2)
    }
#undef C3PT_BV
    *err = hipErrorInvalidValue;
    return 0;
}

template <template <typename, int, int> class ProdT>
int batch_dispatch(int mode, int mt, int variant, const BatchGrid* bg, int n_wg, hipStream_t st, hipError_t* err) {
    *err = hipSuccess;
    switch (mode) {
        case kModeF32: return batch_variant<ProdT, NativeCons, float>(mt, variant, bg, n_wg, st, err);
        case kModeSplitBF16: return batch_variant<ProdT, SplitCons, __bf16>(mt, variant, bg, n_wg, st, err);
        case kModeSplitF16: return batch_variant<ProdT, SplitCons, _Float16>(mt, variant, bg, n_wg, st, err);
        default: *err = hipErrorInvalidValue; return 0;
    }
}

// MTMAX (row tiles of the layout) of a momentum-tile class.
inline int class_mtmax(int mt) { return mt <= 4 ? 4 : mt <= 8 ? 8 : mt <= 12 ? 12 : 16; }

template <template <typename, int, int> class ProdT>
hipError_t dispatch(int mode, int mt, int variant, const ProjGrid& pg,
                    const typename ProdT<float, 16, 256>::Args& a, hipStream_t st) {
    switch (mode) {
        case kModeF64:
            if (mt <= 4 && variant == 0) return launch_cons<NativeCons<double, 16, 4, 1, 3, 1>, ProdT>(pg, a, st);
            return hipErrorInvalidValue;
        case kModeF32:
            return launch_variant<ProdT, NativeCons, float>(mt, variant, pg, a, st);
        case kModeSplitBF16:
            return launch_variant<ProdT, SplitCons, __bf16>(mt, variant, pg, a, st);
        case kModeSplitF16:
            return launch_variant<ProdT, SplitCons, _Float16>(mt, variant, pg, a, st);
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace c3pt
