// Factored momentum projection for gfx950 (MI355X).
//
// The phase of Eqs. (9)-(10) factorizes over the three directions,
//   exp(sigma 2 pi i k.x / L) = w1^(k1 x1) w2^(k2 x2) w3^(k3 x3),  w_j = exp(sigma 2 pi i / L_j),
// so the projection of the contracted tensor P(x, c) onto a momentum list runs
// as three nested partial sums instead of one dense (momenta x sites) GEMM:
//   stage 1, per x1 row:    R1[a][c]  = sum_x1 w1^(K1[a] x1) P(x, c)   a over the distinct k1
//   stage 2, per x3 plane:  R2[b][c] += w2^(k2_b x2) R1[a(b)][c]       b over the distinct (k1, k2)
//   stage 3, per chunk:     S[m][c]  += w3^(k3_m x3) R2[b(m)][c]       m over the momenta
// Stage 1 is a complex GEMM on the matrix cores (16 rows = 8 k1 values x
// (re, im), K = (site, re/im) of a row segment); stages 2 and 3 are small
// complex multiply-adds.  For a ball of momenta (|k|^2 <= 9: 7 k1 values,
// 29 (k1, k2) pairs) this is about a tenth of the dense GEMM's arithmetic, and
// no phase table is read: the workgroup keeps the three root-of-unity tables
// in LDS.
//
// One workgroup owns one column block and one chunk of x3 planes.  Tiles are
// KT consecutive sites of one x1 row (rows shorter than KT, or the last
// segment of a row, contribute zeros beyond the row end).  Twelve waves, one
// per 16-column tile; the producers (c3pt_producers.h) are the ones of the
// dense kernels.  S is held in registers: thread t owns column t % 192 and the
// momenta m = t / 192 + 4 i.  The chunk sums are written in the accumulator
// type and reduced in FP64 with the source factor, as for the dense kernels.
#pragma once

#include <type_traits>

#include "c3pt_fac_prod.h"

namespace c3pt {

template <typename R> struct FacLimits;
template <> struct FacLimits<float> {
    static constexpr int kPairs = kFacMaxPairsF32;
    static constexpr int kOut = kMaxMomGroupF32 / 4;
    static constexpr int kSegs = 4;            // row segments whose A operands are kept in LDS
};
template <> struct FacLimits<double> {
    static constexpr int kPairs = kFacMaxPairsF64;
    static constexpr int kOut = kMaxMomGroupF64 / 4;
    static constexpr int kSegs = 1;
};

template <typename R, int KT>
struct FacSmem {
    static constexpr int PST = 2 * KT + 2;     // slot stride of P (R elements); = 2 mod 32
    static constexpr int KS = 2 * KT / 4;      // MFMA K steps per tile
    static constexpr int kA1 = FacLimits<R>::kSegs > 2 ? FacLimits<R>::kSegs : 2;
    R P[kBlockCols * PST];                     // P[slot][2 * site + re/im], slots owned by waves
    // stage-1 A operands [slot][K step][lane]: every segment of a row when they
    // fit (filled once per work item), else two slots alternating by tile
    R A1[kA1][KS][64];
    C2<R> R2[FacLimits<R>::kPairs][kBlockCols];   // stage-2 sums of a plane, gathered for stage 3
    C2<R> coef2[2][FacLimits<R>::kPairs + kFacMaxBPerA];   // w2^(k2_b x2), by row parity, zero-padded
    C2<R> root[3][kMaxL];
    FactorPlan plan;
};

// Stage-1 A row r of a 16-row tile -> (k1 index a, part re/im), chosen so that
// both accumulator layouts hold (re, im) of a = 2g, 2g+1 in registers (0,1), (2,3).
template <typename R>
__device__ __forceinline__ void fac_row(int r, int& a, int& part) {
    if (Mfma<R>::kRowsByRegister) {
        part = (r >> 2) & 1;
        a = 2 * (r & 3) + (r >> 3);
    } else {
        part = r & 1;
        a = r >> 1;
    }
}

// Plan into LDS, root tables.  Ends with a barrier.
template <typename R, int KT>
__device__ __forceinline__ void fac_setup(FacSmem<R, KT>& sm, const FactorPlan* gplan, int tid, int NT) {
    const int* src = (const int*)gplan;
    int* dst = (int*)&sm.plan;
    for (int i = tid; i < (int)(sizeof(FactorPlan) / sizeof(int)); i += NT) dst[i] = src[i];
    const int sigma = gplan->sigma;
    for (int i = tid; i < 3 * kMaxL; i += NT) {
        const int j = i / kMaxL, x = i % kMaxL;
        const int L = gplan->L[j];
        C2<R> w = {0, 0};
        if (x < L) {
            double s, c;
            sincospi(2.0 * (double)x / (double)L, &s, &c);
            w = {(R)c, (R)(sigma * s)};
        }
        sm.root[j][x] = w;
    }
    __syncthreads();
}

// Stage-1 A operand of the row segment starting at x1 = s: value for (K step
// ks, lane al).  Zero for sites past the row end (their P slots hold copies).
template <typename R, int KT>
__device__ __forceinline__ R fac_a1(const FacSmem<R, KT>& sm, int s, int ks, int al, int L1, float inv1) {
    int a, part;
    fac_row<R>(al & 15, a, part);
    const int kk = al >> 4;
    const int j = 2 * ks + (kk >> 1), comp = kk & 1;
    if (a >= sm.plan.n1 || s + j >= L1) return (R)0;
    const C2<R> w = sm.root[0][mod_small(sm.plan.k1[a] * (s + j), L1, inv1)];
    return part == 0 ? (comp == 0 ? w.x : -w.y) : (comp == 0 ? w.y : w.x);
}

// Partial-sum element type.
template <typename R> using Part2 = typename std::conditional<sizeof(R) == 8, double2, float2>::type;

// Orders this wave's LDS writes before its later LDS reads of other lanes'
// data (no workgroup barrier: the data never leaves the wave).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over the tiles of planes [p0, p1).  ACC: into out (thread-owned
// momenta), written by fac_write at the end.  Otherwise every plane's sums are
// added into the chunk's partial sums in global memory (written at the first
// plane, read back and added at the next ones; each element is owned by one
// thread of one workgroup, so the order is fixed); out is unused.
//
// Software pipeline, one workgroup barrier per tile T:
//   contract(T) -> P (own slots) | stage(T+1) -> buf[(T+1)&1] | loads of T+2 |
//   stage 1 (MFMA on own slots) | stage 2 at row ends | barrier | stage 3 at plane ends
// The per-site buffers, the row coefficients and (for long rows) the A
// operands are written one tile ahead into the half not being read.  The
// contraction inputs are held in three register sets (tiles T, T+1, T+2) so
// that their loads have more than a tile to arrive.  PHASE staggers the
// loads of tile T+2 over the waves: before the contraction (1), in its middle
// (2, producers that split it) or after it (0), so that the address units
// work while part of the workgroup computes, instead of all waves issuing
// their loads at once.
template <typename R, int KT, bool ACC, int PHASE, class Prod>
__device__ __forceinline__ void fac_loop(const typename Prod::Ctx& ctx, const TileGeom& tg, FacSmem<R, KT>& sm,
                                         typename Prod::Buf (&buf)[2], int p0, int p1,
                                         C2<R> (&out)[FacLimits<R>::kOut], void* partial, int n_colblocks,
                                         int cb, int chunk, int tid) {
    using MF = Mfma<R>;
    using acc_t = typename MF::acc_t;
    using S = typename Prod::S;
    constexpr int KS = FacSmem<R, KT>::KS;
    constexpr int PST = FacSmem<R, KT>::PST;
    constexpr int NT = kFacThreads;
    const int L1 = tg.L1, L2 = tg.L2, L3 = tg.L3;
    const float inv1 = 1.0f / (float)L1, inv2 = 1.0f / (float)L2, inv3 = 1.0f / (float)L3;
    const int nseg = (L1 + KT - 1) / KT;
    const bool a1_all = nseg <= FacLimits<R>::kSegs;
    const int n_tiles = (p1 - p0) * L2 * nseg;
    if (n_tiles <= 0) return;
    const int lane = tid & 63, wave = tid >> 6, g = lane >> 4;
    const int slot = 16 * wave + (lane & 15);     // this lane's MFMA column
    int lcol;                                     // its column in the block
    {
        int X, r;
        S::of_slot(slot, X, r);
        lcol = Prod::col(X, r);
    }
    const int n_mom = sm.plan.n_mom, n12 = sm.plan.n12;
    const int nbmax = __builtin_amdgcn_readfirstlane(sm.plan.nbmax);
    // stage-2 ownership: k1 indices 2g, 2g+1 of column lcol, their pairs in registers
    int bs[2], nb[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int a = 2 * g + h;
        bs[h] = a < sm.plan.n1 ? sm.plan.bstart[a] : 0;
        nb[h] = a < sm.plan.n1 ? sm.plan.bstart[a + 1] - bs[h] : 0;
    }
    C2<R> r2[2][kFacMaxBPerA];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < kFacMaxBPerA; ++i) r2[h][i] = C2<R>{0, 0};
    // stage-3 ownership
    const int c3 = tid % kBlockCols, q3 = tid / kBlockCols;

    // Tile positions advance by counting (no division per tile): segment,
    // row of the chunk (x2, x3) and row number (its parity picks the row
    // coefficients).  Uniform, so they stay in scalar registers.
    struct TilePos {
        int seg, x2, x3, row;
    };
    auto advance = [&](TilePos q) {
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
    const int jt = tid % KT;
    auto site_of = [&](const TilePos& q) {
        RowSite rs;
        rs.x1 = min(q.seg * KT + jt, L1 - 1);
        rs.x2 = q.x2;
        rs.x3 = q.x3;
        rs.n = rs.x1 + L1 * (q.x2 + L2 * q.x3);
        Prod::prepare(ctx, rs);
        return rs;
    };
    auto fill_a1 = [&](int slot_a, int s) {
        for (int e = tid; e < KS * 64; e += NT) sm.A1[slot_a][e >> 6][e & 63] = fac_a1<R, KT>(sm, s, e >> 6, e & 63, L1, inv1);
    };
    auto fill_coef2 = [&](int par, int x2) {
        for (int b = tid; b < n12 + kFacMaxBPerA; b += NT)
            sm.coef2[par][b] = b < n12 ? sm.root[1][mod_small(sm.plan.k2[b] * x2, L2, inv2)] : C2<R>{0, 0};
    };
    FacPut<R, KT> put{sm.P, PST};
    typename Prod::Pre pre;
    typename Prod::Main m0, m1, m2;

    // prologue: tile 0 staged, contraction inputs of tiles 0 and 1 and
    // per-site inputs of tile 1 in flight
    if (a1_all) {
        for (int e = tid; e < nseg * KS * 64; e += NT) {
            const int seg = e / (KS * 64), rem = e % (KS * 64);
            sm.A1[seg][rem >> 6][rem & 63] = fac_a1<R, KT>(sm, seg * KT, rem >> 6, rem & 63, L1, inv1);
        }
    } else {
        fill_a1(0, 0);
    }
    // positions of tiles T, T+1, T+2 (the last tile again past the end)
    TilePos pa = {0, 0, p0, 0};
    TilePos pb = n_tiles > 1 ? advance(pa) : pa;
    TilePos pc = n_tiles > 2 ? advance(pb) : pb;
    {
        const RowSite rs0 = site_of(pa);
        fill_coef2(0, rs0.x2);
        // same issue order as the loop (per-site inputs, then contraction inputs)
        Prod::load_pre(ctx, tg, rs0, pre, tid);
        Prod::load_main(ctx, tg, rs0, m0, tid);
        Prod::stage(ctx, pre, buf[0], tid);
        const RowSite rs1 = site_of(pb);
        Prod::load_pre(ctx, tg, rs1, pre, tid);
        Prod::load_main(ctx, tg, rs1, m1, tid);
    }
    acc_t r1 = acc_t{0, 0, 0, 0};
    __syncthreads();

    // mc holds tile T's contraction inputs, mn receives those of tile T+2
    auto step = [&](int T, typename Prod::Main& mc, typename Prod::Main& mn) {
        const int par = T & 1;
        const int seg = pa.seg, x2 = pa.x2, x3 = pa.x3, row = pa.row;
        const bool row_end = (seg == nseg - 1);
        const bool plane_end = row_end && x2 == L2 - 1;
        // tile T+2 (the last tile again past the end: always in bounds)
        const RowSite rs2 = site_of(pc);
        if (PHASE == 1) Prod::load_main(ctx, tg, rs2, mn, tid);
        // contraction of tile T into this wave's slots
        if constexpr (PHASE == 2) {
            Prod::template contract_part<0, 1>(ctx, mc, buf[par], put, tid);
            Prod::load_main(ctx, tg, rs2, mn, tid);
            Prod::template contract_part<1, 4>(ctx, mc, buf[par], put, tid);
        } else {
            Prod::contract(ctx, mc, buf[par], put, tid);
        }
        // tile T+1: per-site buffer, row coefficients, A operands
        if (T + 1 < n_tiles) {
            Prod::stage(ctx, pre, buf[par ^ 1], tid);
            if (pb.seg == 0) fill_coef2(pb.row & 1, pb.x2);
            if (!a1_all) fill_a1(par ^ 1, pb.seg * KT);
        }
        Prod::load_pre(ctx, tg, rs2, pre, tid);
        if (PHASE == 0) Prod::load_main(ctx, tg, rs2, mn, tid);
        wave_lds_sync();
        // stage 1 on this wave's own slots
        const int sa = a1_all ? seg : par;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) r1 = MF::mac(sm.A1[sa][ks][lane], sm.P[slot * PST + 4 * ks + g], r1);
        if (row_end) {
            // stage 2, in registers
            const C2<R>* cf = sm.coef2[row & 1];
            if constexpr (sizeof(R) == 4) {
                // every register of both slots is updated: the coefficient
                // table is zero-padded by kFacMaxBPerA entries, so all reads
                // are in bounds, and registers beyond a lane's pairs are never
                // gathered.  No branch between the reads: all are in flight
                // at once.
                C2<R> cw[2][kFacMaxBPerA];
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int i = 0; i < kFacMaxBPerA; ++i) cw[h][i] = cf[bs[h] + i];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const C2<R> v = h == 0 ? C2<R>{r1[0], r1[1]} : C2<R>{r1[2], r1[3]};
#pragma unroll
                    for (int i = 0; i < kFacMaxBPerA; ++i) r2[h][i] = cfma(r2[h][i], cw[h][i], v);
                }
            } else {
                // FP64: twice the registers per coefficient; the first nbmax
                // registers are updated one pair at a time (a uniform bound)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const C2<R> v = h == 0 ? C2<R>{r1[0], r1[1]} : C2<R>{r1[2], r1[3]};
#pragma unroll
                    for (int i = 0; i < kFacMaxBPerA; ++i)
                        if (i < nbmax) r2[h][i] = cfma(r2[h][i], cf[bs[h] + i], v);
                }
            }
            r1 = acc_t{0, 0, 0, 0};
            if (plane_end) {
                // plane x3 done: gather the stage-2 sums for stage 3
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    C2<R>* dst = &sm.R2[bs[h]][lcol];   // pair i at dst[i * kBlockCols]
#pragma unroll
                    for (int i = 0; i < kFacMaxBPerA; ++i) {
                        if (i < nb[h]) dst[i * kBlockCols] = r2[h][i];
                        r2[h][i] = C2<R>{0, 0};
                    }
                }
            }
        }
        __syncthreads();
        if (plane_end) {
            // stage 3
            if (ACC) {
#pragma unroll
                for (int i = 0; i < FacLimits<R>::kOut; ++i) {
                    const int m = q3 + 4 * i;
                    if (m < n_mom) {
                        const int b = sm.plan.pair_of_m[m];
                        const C2<R> w = sm.root[2][mod_small(sm.plan.k3[m] * x3, L3, inv3)];
                        out[i] = cfma(out[i], w, sm.R2[b][c3]);
                    }
                }
            } else {
                Part2<R>* part = (Part2<R>*)partial;
                const size_t base = ((size_t)chunk * n_colblocks + cb) * (size_t)n_mom;
                const bool first = (x3 == p0);
                for (int m = q3; m < n_mom; m += 4) {
                    const int b = sm.plan.pair_of_m[m];
                    const C2<R> w = sm.root[2][mod_small(sm.plan.k3[m] * x3, L3, inv3)];
                    C2<R> v = cmul(w, sm.R2[b][c3]);
                    Part2<R>& dst = part[(base + m) * kBlockCols + c3];
                    if (!first) {
                        const Part2<R> o = dst;
                        v.x += o.x;
                        v.y += o.y;
                    }
                    dst = Part2<R>{v.x, v.y};
                }
            }
            // R2 is gathered again only after this barrier
            __syncthreads();
        }
        pa = pb;
        pb = pc;
        if (T + 3 < n_tiles) pc = advance(pc);
    };
    // three register sets in turn, without a branch between the steps (the
    // load counters are then tracked exactly), the last one or two tiles after
    int T = 0;
    for (; T + 2 < n_tiles; T += 3) {
        step(T, m0, m2);
        step(T + 1, m1, m0);
        step(T + 2, m2, m1);
    }
    if (T < n_tiles) step(T, m0, m2);
    if (T + 1 < n_tiles) step(T + 1, m1, m0);
}

// Producers whose contraction splits into parts (contract_part<X0, X1>).
template <class Prod, class = void>
struct FacSplit : std::false_type {};
template <class Prod>
struct FacSplit<Prod, std::void_t<decltype(Prod::kSplitContract)>> : std::integral_constant<bool, Prod::kSplitContract> {};

// Load phase of a wave: waves 4..7 (one on each SIMD) issue the loads of tile
// T+2 before their contraction, waves 8..11 in its middle when the producer
// splits it, the others after it.  Uniform per wave; every form passes the
// same workgroup barriers in the same order.
template <class Prod>
__device__ __forceinline__ int fac_load_phase(int tid) {
    const int g = __builtin_amdgcn_readfirstlane(tid >> 6) / 4;
    return g == 1 ? 1 : (g == 2 && FacSplit<Prod>::value ? 2 : 0);
}

// Runs the tile loop in the form of the wave's load phase.
template <typename R, int KT, bool ACC, class Prod, class... A>
__device__ __forceinline__ void fac_loop_phased(int tid, A&&... args) {
    const int ph = fac_load_phase<Prod>(tid);
    if (ph == 1) {
        fac_loop<R, KT, ACC, 1, Prod>(args..., tid);
    } else {
        if constexpr (FacSplit<Prod>::value) {
            if (ph == 2) {
                fac_loop<R, KT, ACC, 2, Prod>(args..., tid);
                return;
            }
        }
        fac_loop<R, KT, ACC, 0, Prod>(args..., tid);
    }
}

template <typename R>
__device__ __forceinline__ void fac_write(void* partial, int n_colblocks, int n_mom, int chunk, int cb,
                                          const C2<R> (&out)[FacLimits<R>::kOut], int tid) {
    using P2 = Part2<R>;
    P2* part = (P2*)partial;
    const int c = tid % kBlockCols, q = tid / kBlockCols;
    const size_t base = ((size_t)chunk * n_colblocks + cb) * (size_t)n_mom;
#pragma unroll
    for (int i = 0; i < FacLimits<R>::kOut; ++i) {
        const int m = q + 4 * i;
        if (m < n_mom) part[(base + m) * kBlockCols + c] = P2{out[i].x, out[i].y};
    }
}

template <typename R, int KT, bool ACC, template <typename, int, int> class ProdT>
__global__ void __launch_bounds__(kFacThreads, 1)
fac_kernel(ProjGrid pg, typename ProdT<R, KT, kFacThreads>::Args pa) {
    using Prod = ProdT<R, KT, kFacThreads>;
    __shared__ FacSmem<R, KT> sm;
    __shared__ typename Prod::Buf buf[2];
    const int tid = threadIdx.x;
    // work item (within, share, chunk), chunk outermost; consecutive items run
    // on one XCD: those of one (share, chunk) read the same input slice, and
    // neighbouring shares (timeslices) of a chunk read each other's slice as
    // the derivative's t +- 1 neighbours while it is still in that XCD's L2
    const int nw = gridDim.x, w = blockIdx.x;
    const int full = (nw / 8) * 8;
    const int item = (w < full) ? (w % 8) * (nw / 8) + w / 8 : w;
    const int within = item % pg.n_per_share;
    const int rest = item / pg.n_per_share;
    const int share = rest % pg.n_share;
    const int chunk = rest / pg.n_share;
    const int cb = Prod::colblock(pa, share, within);
    const typename Prod::Ctx ctx = Prod::resolve(pa, pg.V3, cb);
    TileGeom tg;
    tg.V3 = pg.V3;
    tg.L1 = pa.L[0];
    tg.L2 = pa.L[1];
    tg.L3 = pa.L[2];
    tg.inv1 = 1.0f / (float)tg.L1;
    tg.inv12 = 1.0f / (float)(tg.L1 * tg.L2);
    tg.row = tg.x1 = tg.x2 = tg.x3 = 0;
    fac_setup<R, KT>(sm, (const FactorPlan*)pg.phase, tid, kFacThreads);
    C2<R> out[FacLimits<R>::kOut];
    if (ACC) {
#pragma unroll
        for (int i = 0; i < FacLimits<R>::kOut; ++i) out[i] = C2<R>{0, 0};
    }
    const int p0 = chunk * pg.chunk_planes;
    const int p1 = min(tg.L3, p0 + pg.chunk_planes);
    fac_loop_phased<R, KT, ACC, Prod>(tid, ctx, tg, sm, buf, p0, p1, out, pg.partial, pg.n_colblocks, cb, chunk);
    if (ACC) fac_write<R>(pg.partial, pg.n_colblocks, pg.n_mom, chunk, cb, out, tid);
}

// Form for batches and serving: one workgroup per (job, column block, plane
// chunk) item of the launch's item list; job.phase is the job's FactorPlan,
// job.chunk_sites the x3 planes per chunk, job.n_chunks the chunks.  The
// hardware hands out workgroups in order as CUs free up, which balances the
// uneven items as a work queue would; consecutive items (the same input slice
// and chunk) are mapped onto one XCD, so they share its L2.
template <typename R, int KT, template <typename, int, int> class ProdT>
__global__ void __launch_bounds__(kFacThreads, 1) fac_batch_kernel(BatchGrid bg) {
    using Prod = ProdT<R, KT, kFacThreads>;
    __shared__ FacSmem<R, KT> sm;
    __shared__ typename Prod::Buf buf[2];
    const int tid = threadIdx.x;
    const int nw = gridDim.x, w = blockIdx.x;
    const int full = (nw / 8) * 8;
    const int it = (w < full) ? (w % 8) * (nw / 8) + w / 8 : w;
    const int4 item = bg.items[it];
    const BatchJob& job = bg.jobs[item.x];
    const int cb = item.y;
    const typename Prod::Ctx ctx = Prod::resolve(job, job.V3, cb);
    TileGeom tg;
    tg.V3 = job.V3;
    tg.L1 = job.L[0];
    tg.L2 = job.L[1];
    tg.L3 = job.L[2];
    tg.inv1 = 1.0f / (float)tg.L1;
    tg.inv12 = 1.0f / (float)(tg.L1 * tg.L2);
    tg.row = tg.x1 = tg.x2 = tg.x3 = 0;
    fac_setup<R, KT>(sm, (const FactorPlan*)job.phase, tid, kFacThreads);
    C2<R> out[FacLimits<R>::kOut];   // not used by the plane-chunk form
    const int p0 = item.z * job.chunk_sites;
    const int p1 = min(tg.L3, p0 + job.chunk_sites);
    fac_loop_phased<R, KT, false, Prod>(tid, ctx, tg, sm, buf, p0, p1, out, job.partial, job.n_colblocks, cb, item.z);
}

// Launches one workgroup per item (bg->n_items); with bg == nullptr only the
// occupancy (workgroups per CU) is returned.
template <typename R, int KT, template <typename, int, int> class ProdT>
int fac_batch_kt(const BatchGrid* bg, hipStream_t st, hipError_t* err) {
    *err = hipSuccess;
    if (bg) {
        hipLaunchKernelGGL((fac_batch_kernel<R, KT, ProdT>), dim3(bg->n_items), dim3(kFacThreads), 0, st, *bg);
        *err = hipGetLastError();
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fac_batch_kernel<R, KT, ProdT>, kFacThreads, 0) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

// Launch in the form the variant selects: 32-site tiles (kBatchFacKT32) only
// where the producer allows them.
template <template <typename, int, int> class ProdT, bool kAllow32>
int fac_batch(int variant, const BatchGrid* bg, hipStream_t st, hipError_t* err) {
    if constexpr (kAllow32) {
        if (variant & kBatchFacKT32) return fac_batch_kt<float, 32, ProdT>(bg, st, err);
    }
    return fac_batch_kt<float, 16, ProdT>(bg, st, err);
}

template <typename R, int KT, bool ACC, template <typename, int, int> class ProdT>
hipError_t launch_fac_kt(const ProjGrid& pg, const typename ProdT<R, KT, kFacThreads>::Args& a, hipStream_t st) {
    hipLaunchKernelGGL((fac_kernel<R, KT, ACC, ProdT>), dim3(pg.n_share * pg.n_per_share * pg.n_chunks), dim3(kFacThreads), 0,
                       st, pg, a);
    return hipGetLastError();
}

// FP32: 32-site tiles when whole rows split into them and the producer keeps
// its registers at that size (kAllow32), else 16; FP64: 16.  acc selects the
// form that sums a chunk's planes in registers.
template <template <typename, int, int> class ProdT, bool kAllow32, class Args>
hipError_t launch_fac(bool f64, bool acc, const ProjGrid& pg, const Args& a, hipStream_t st) {
    if (f64) return acc ? launch_fac_kt<double, 16, true, ProdT>(pg, a, st) : launch_fac_kt<double, 16, false, ProdT>(pg, a, st);
    if constexpr (kAllow32) {
        if (a.L[0] % 32 == 0)
            return acc ? launch_fac_kt<float, 32, true, ProdT>(pg, a, st) : launch_fac_kt<float, 32, false, ProdT>(pg, a, st);
    }
    return acc ? launch_fac_kt<float, 16, true, ProdT>(pg, a, st) : launch_fac_kt<float, 16, false, ProdT>(pg, a, st);
}

}  // namespace c3pt
