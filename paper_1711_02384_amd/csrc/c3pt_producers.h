// Producers of libc3pt: contract one tile of KT sites into P[col][site] for
// one 192-column block.  A column block is first resolved into a context of
// plain pointers (Ctx, once per work item); then, per tile:
//   load(...)  -> registers (Regs), issued before the MFMA loop of the previous tile
//   store(...) -> contraction from registers (+ LDS staging) into the sink
// Every thread keeps one site j = tid % KT of the tile.  Sites j >= nsite
// contribute zeros.
#pragma once

#include "c3pt_device.h"

namespace c3pt {

template <int N, int NT>
struct PerThread {
    static constexpr int value = (N + NT - 1) / NT;
};

// Element idx of a field, or zero when !ok, without a branch: the load always
// runs (at element 0 when it is not wanted) and the value is selected after.
// Indices are unsigned 32-bit: 144 * V3 < 2^32 for every allowed extent.
template <typename R>
__device__ __forceinline__ C2<R> ld_or_zero(const C2<R>* p, unsigned idx, bool ok) {
    const C2<R> v = p[ok ? idx : 0u];
    return ok ? v : C2<R>{0, 0};
}

// ---------------------------------------------------------------------------
// Meson spectator, Eq. (9):
//   P[(b',a',a,c)] = g[b'] g[a'] g[a] sum_c' eta[(b',c')] conj(G[(a',c')][(a,c)])
// Column block cb = noise.  Task (site j, q = a'*12 + a*3 + c) computes the
// four b' columns from three propagator entries.
// ---------------------------------------------------------------------------
template <typename R, int KT, int NT>
struct MesonSpecProducer {
    using Args = MesonSpecArgs;
    static_assert(NT % KT == 0, "every thread keeps one site of the tile");
    static constexpr int kV = PerThread<12 * KT, NT>::value;
    static constexpr int kT = PerThread<48 * KT, NT>::value;
    struct Ctx {
        const C2<R>* G;
        const C2<R>* eta;   // this noise vector
    };
    struct Regs {
        C2<R> v[kV];
        C2<R> g[kT][3];
    };
    struct Smem {
        C2<R> v[12][KT];
    };
    static __device__ __forceinline__ int colblock(const Args&, int, int within) { return within; }
    static __device__ __forceinline__ Ctx resolve(const Args& a, int V3, int cb) {
        return Ctx{(const C2<R>*)a.G, (const C2<R>*)a.eta + (size_t)cb * 12 * V3};
    }
    static __device__ __forceinline__ Ctx resolve(const BatchJob& b, int V3, int cb) {
        return Ctx{(const C2<R>*)b.G, (const C2<R>*)b.eta + (size_t)cb * 12 * V3};
    }
    static __device__ __forceinline__ void load(const Ctx& c, const TileGeom& tg, int t0, int nsite, Regs& rg,
                                                int tid) {
        const unsigned V3 = (unsigned)tg.V3;
        const int j = tid % KT;
        const bool site_ok = j < nsite;
        const unsigned n = (unsigned)(t0 + j);
#pragma unroll
        for (int i = 0; i < kV; ++i) {
            const int e = tid + i * NT, A = e / KT;
            rg.v[i] = ld_or_zero(c.eta, (unsigned)A * V3 + n, e < 12 * KT && site_ok);
        }
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int e = tid + i * NT, q = e / KT;
            const int ap = q / 12, rem = q % 12;
            const bool ok = e < 48 * KT && site_ok;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                rg.g[i][cc] = ld_or_zero(c.G, (unsigned)((3 * ap + cc) * 12 + rem) * V3 + n, ok);
        }
    }
    template <class Sink>
    static __device__ __forceinline__ void store(const Ctx&, const TileGeom&, int, int, const Regs& rg, Smem& sm,
                                                 Sink& sink, int tid) {
        const int j = tid % KT;
#pragma unroll
        for (int i = 0; i < kV; ++i) {
            const int e = tid + i * NT, A = e / KT;
            if (e < 12 * KT) sm.v[A][j] = (A >= 6) ? C2<R>{-rg.v[i].x, -rg.v[i].y} : rg.v[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int e = tid + i * NT, q = e / KT;
            if (e >= 48 * KT) continue;
            const int ap = q / 12, al = (q % 12) / 3;
            const R sg = g5<R>(ap) * g5<R>(al);
#pragma unroll
            for (int bp = 0; bp < 4; ++bp) {
                C2<R> p = cmulc(sm.v[3 * bp][j], rg.g[i][0]);
                p = cadd(p, cmulc(sm.v[3 * bp + 1][j], rg.g[i][1]));
                p = cadd(p, cmulc(sm.v[3 * bp + 2][j], rg.g[i][2]));
                sink.put(bp * 48 + q, j, cscale(p, sg));
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Nucleon-type spectator with epsilon tensors at sink and source.  Column
// block cb = noise * 16 + (a1' * 4 + a1); columns (a2', a2, b', c').
//   P = g[b'] sum_c eta[(b',c)] Q[c][c'],
//   Q[c][c'] = sum eps_{abc} eps_{a'b'c'} G1[(a1',a)][(a1,a')] G2[(a2',b)][(a2,b')]
// Task (site j, q = a2'*4 + a2) forms Q from nine G2 entries and the G1 block.
// ---------------------------------------------------------------------------
template <typename R, int KT, int NT>
struct BaryonSpecProducer {
    using Args = BaryonSpecArgs;
    static_assert(NT % KT == 0, "every thread keeps one site of the tile");
    static constexpr int kV = PerThread<21 * KT, NT>::value;
    static constexpr int kT = PerThread<16 * KT, NT>::value;
    struct Ctx {
        const C2<R>* G1;
        const C2<R>* G2;
        const C2<R>* eta;   // this noise vector
        int a1p, a1;
    };
    struct Regs {
        C2<R> v[kV];
        C2<R> g2[kT][9];
    };
    struct Smem {
        C2<R> v[12][KT];
        C2<R> g1[9][KT];
    };
    static __device__ __forceinline__ int colblock(const Args&, int, int within) { return within; }
    static __device__ __forceinline__ Ctx make(const void* G1, const void* G2, const void* eta, int V3, int cb) {
        const int blk = cb & 15;
        return Ctx{(const C2<R>*)G1, (const C2<R>*)G2, (const C2<R>*)eta + (size_t)(cb >> 4) * 12 * V3, blk >> 2,
                   blk & 3};
    }
    static __device__ __forceinline__ Ctx resolve(const Args& a, int V3, int cb) {
        return make(a.G1, a.G2, a.eta, V3, cb);
    }
    static __device__ __forceinline__ Ctx resolve(const BatchJob& b, int V3, int cb) {
        return make(b.G, b.G2, b.eta, V3, cb);
    }
    static __device__ __forceinline__ void load(const Ctx& c, const TileGeom& tg, int t0, int nsite, Regs& rg,
                                                int tid) {
        const unsigned V3 = (unsigned)tg.V3;
        const int j = tid % KT;
        const bool site_ok = j < nsite;
        const unsigned n = (unsigned)(t0 + j);
#pragma unroll
        for (int i = 0; i < kV; ++i) {
            const int e = tid + i * NT, A = e / KT;
            const bool ok = e < 21 * KT && site_ok;
            // entries 0..11: the noise vector; 12..20: the G1 block of (a1', a1)
            const bool is_eta = A < 12;
            const int cc = is_eta ? 0 : A - 12;
            const C2<R>* base = is_eta ? c.eta : c.G1;
            const unsigned idx = is_eta ? (unsigned)A * V3 + n
                                        : (unsigned)((3 * c.a1p + cc / 3) * 12 + 3 * c.a1 + cc % 3) * V3 + n;
            rg.v[i] = ld_or_zero(base, idx, ok);
        }
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int e = tid + i * NT, q = e / KT;
            const int a2p = q >> 2, a2 = q & 3;
            const bool ok = e < 16 * KT && site_ok;
#pragma unroll
            for (int cc = 0; cc < 9; ++cc)
                rg.g2[i][cc] = ld_or_zero(c.G2, (unsigned)((3 * a2p + cc / 3) * 12 + 3 * a2 + cc % 3) * V3 + n, ok);
        }
    }
    template <class Sink>
    static __device__ __forceinline__ void store(const Ctx&, const TileGeom&, int, int, const Regs& rg, Smem& sm,
                                                 Sink& sink, int tid) {
        const int j = tid % KT;
#pragma unroll
        for (int i = 0; i < kV; ++i) {
            const int e = tid + i * NT, A = e / KT;
            if (e >= 21 * KT) continue;
            if (A < 12) sm.v[A][j] = (A >= 6) ? C2<R>{-rg.v[i].x, -rg.v[i].y} : rg.v[i];
            else sm.g1[A - 12][j] = rg.v[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int e = tid + i * NT, q = e / KT;
            if (e >= 16 * KT) continue;
            C2<R> g1[9];
#pragma unroll
            for (int cc = 0; cc < 9; ++cc) g1[cc] = sm.g1[cc][j];
            const C2<R>* g2 = rg.g2[i];
            // Q[c][c'] with (a, b) = (c+1, c+2) (+) and (c+2, c+1) (-), same for primes.
            C2<R> Q[9];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int ca = (c + 1) % 3, cb2 = (c + 2) % 3;
#pragma unroll
                for (int cp = 0; cp < 3; ++cp) {
                    const int pa = (cp + 1) % 3, pb = (cp + 2) % 3;
                    C2<R> t = cmul(g1[ca * 3 + pa], g2[cb2 * 3 + pb]);
                    t = csub(t, cmul(g1[ca * 3 + pb], g2[cb2 * 3 + pa]));
                    t = csub(t, cmul(g1[cb2 * 3 + pa], g2[ca * 3 + pb]));
                    t = cfma(t, g1[cb2 * 3 + pb], g2[ca * 3 + pa]);
                    Q[c * 3 + cp] = t;
                }
            }
#pragma unroll
            for (int bp = 0; bp < 4; ++bp) {
                const C2<R> v0 = sm.v[3 * bp][j], v1 = sm.v[3 * bp + 1][j], v2 = sm.v[3 * bp + 2][j];
#pragma unroll
                for (int cp = 0; cp < 3; ++cp) {
                    C2<R> p = cmul(v0, Q[cp]);
                    p = cfma(p, v1, Q[3 + cp]);
                    p = cfma(p, v2, Q[6 + cp]);
                    sink.put((q * 4 + bp) * 3 + cp, j, p);
                }
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Insertion, Eq. (10).  Column block cb = ((noise * n_tau) + tau) * n_ops + op;
// columns (at, bt, b, c).  op 0: P = sum_c' v[at][c'] G[(bt,c')][(b,c)] with
// v = g[at] conj(s[(at,c')]).  op 1+nu: the covariant derivative is moved onto
// the stochastic vector, t+ = 1/2 v U_nu(y), t- = 1/2 v U_nu(y-nu)^dag, and
// P = sum_d t+[at][d] G(y+nu)[(bt,d)][(b,c)] - t-[at][d] G(y-nu)[(bt,d)][(b,c)].
// Task (site j, q = bt*12 + b*3 + c) computes the four at columns.
// ---------------------------------------------------------------------------
// OPS selects the operators a kernel instantiation handles: 0 both (column
// blocks decide), 1 the local operator only, 2 the derivative operators only.
// Single-kind instantiations keep only the registers of their path.
template <typename R, int KT, int NT, int OPS>
struct InsertionProducerT {
    using Args = InsertionArgs;
    static_assert(NT % KT == 0, "every thread keeps one site of the tile");
    static constexpr int kV = PerThread<12 * KT, NT>::value;
    static constexpr int kT = PerThread<48 * KT, NT>::value;
    struct Ctx {
        const C2<R>* Gf;    // G at y + nu (local op: G(y))
        const C2<R>* Gb;    // G at y - nu
        const C2<R>* s;     // this noise vector at tau
        const C2<R>* U;     // U_nu(y)
        const C2<R>* Um;    // U_nu(y - nu) (time: slice tau - 1)
        int nu;             // -1 for the local operator
    };
    static constexpr bool kFullT = 48 * KT == kT * NT;   // every thread has kT contraction tasks
    static constexpr int kG = OPS == 1 ? 3 : 6;
    static constexpr int kU = OPS == 1 ? 1 : 6;
    struct Regs {
        C2<R> v[kV];        // s entries
        C2<R> u[kV][kU];    // transport task: U(y)[c][d], U(y-nu)[d][c] for c = 0..2
        C2<R> g[kT][kG];    // G entries: local uses [0..2]; derivative (y+nu)[0..2], (y-nu)[3..5]
    };
    struct Smem {
        C2<R> v[12][KT];
        C2<R> tp[12][KT];
        C2<R> tm[12][KT];
    };
    // work items that share a timeslice (share) are adjacent: within = noise * n_ops + op
    // work items of one launch cover operators [a.op_lo, a.op_lo + a.op_cnt)
    static __device__ __forceinline__ int colblock(const Args& a, int share, int within) {
        const int noise = within / a.op_cnt, op = a.op_lo + within % a.op_cnt;
        return (noise * a.n_tau + share) * a.n_ops + op;
    }
    static __device__ __forceinline__ Ctx make(const void* G, const void* Gn, const void* Gp, const void* s,
                                               const void* U, const void* Up, int noise, int op, int V3) {
        Ctx c;
        // -1 for the local operator (kernels that take both kinds branch on it);
        // ops 1 + nu, and 5 + 4 rho + nu of the two-derivative launches
        c.nu = op == 0 ? -1 : ((op - 1) & 3);
        c.s = (const C2<R>*)s + (size_t)noise * 12 * V3;
        if (op == 0) {
            c.Gf = c.Gb = (const C2<R>*)G;
            c.U = c.Um = nullptr;
        } else {
            const int nu = c.nu;
            c.Gf = (const C2<R>*)((nu < 3) ? G : Gn);
            c.Gb = (const C2<R>*)((nu < 3) ? G : Gp);
            c.U = (const C2<R>*)U + (size_t)nu * 9 * V3;
            c.Um = (nu < 3) ? c.U : (const C2<R>*)Up + (size_t)3 * 9 * V3;
        }
        return c;
    }
    static __device__ __forceinline__ Ctx resolve(const Args& a, int V3, int cb) {
        const int op = cb % a.n_ops, rest = cb / a.n_ops;
        const int tl = rest % a.n_tau, noise = rest / a.n_tau;
        return make(a.G[tl], a.Gn[tl], a.Gp[tl], a.s[tl], a.U[tl], a.Up[tl], noise, op, V3);
    }
    static __device__ __forceinline__ Ctx resolve(const BatchJob& b, int V3, int cb) {
        const int op = cb % b.n_ops, rest = cb / b.n_ops;
        const int tl = rest % b.n_tau, noise = rest / b.n_tau;
        const void* const* t = b.tau_ptrs + (size_t)tl * 6;
        return make(t[0], t[1], t[2], t[3], t[4], t[5], noise, op, V3);
    }
    static __device__ __forceinline__ void load(const Ctx& c, const TileGeom& tg, int t0, int nsite, Regs& rg,
                                                int tid) {
        const unsigned V3 = (unsigned)tg.V3;
        const int j = tid % KT;
        const bool site_ok = j < nsite;
        const int n = t0 + j;
#pragma unroll
        for (int i = 0; i < kV; ++i) {
            const int e = tid + i * NT, A = e / KT;
            rg.v[i] = ld_or_zero(c.s, (unsigned)A * V3 + (unsigned)n, e < 12 * KT && site_ok);
        }
        if (OPS == 1 || (OPS == 0 && c.nu < 0)) {
#pragma unroll
            for (int i = 0; i < kT; ++i) {
                const int e = tid + i * NT, q = e / KT;
                const int bt = q / 12, rem = q % 12;
                const bool ok = (kFullT || e < 48 * KT) && site_ok;
#pragma unroll
                for (int cc = 0; cc < 3; ++cc)
                    rg.g[i][cc] = ld_or_zero(c.Gf, (unsigned)((3 * bt + cc) * 12 + rem) * V3 + (unsigned)n, ok);
            }
            return;
        }
        if constexpr (OPS != 1) {
        const int nu = c.nu;
        int np = n, nm = n;
        if (nu < 3) {
            int x1, x2, x3;
            if (tg.row) {
                x1 = tg.x1 + j;
                x2 = tg.x2;
                x3 = tg.x3;
            } else {
                int x0[3];
                site_xyz(tg, t0, x0[0], x0[1], x0[2]);
                site_xyz_from(tg, x0, j, x1, x2, x3);
            }
            np = site_shift_xyz(tg, x1, x2, x3, nu, +1);
            nm = site_shift_xyz(tg, x1, x2, x3, nu, -1);
            if (!site_ok) np = nm = t0;
        }
        // transport tasks (q = at*3 + d, site j): links at y and y - nu
#pragma unroll
        for (int i = 0; i < kV; ++i) {
            const int e = tid + i * NT, q = e / KT, d = q % 3;
            const bool ok = e < 12 * KT && site_ok;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                rg.u[i][cc] = ld_or_zero(c.U, (unsigned)(cc * 3 + d) * V3 + (unsigned)n, ok);
                rg.u[i][3 + cc] = ld_or_zero(c.Um, (unsigned)(d * 3 + cc) * V3 + (unsigned)nm, ok);
            }
        }
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int e = tid + i * NT, q = e / KT;
            const int bt = q / 12, rem = q % 12;
            const bool ok = (kFullT || e < 48 * KT) && site_ok;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const unsigned plane = (unsigned)((3 * bt + d) * 12 + rem) * V3;
                rg.g[i][d] = ld_or_zero(c.Gf, plane + (unsigned)np, ok);
                rg.g[i][3 + d] = ld_or_zero(c.Gb, plane + (unsigned)nm, ok);
            }
        }
        }
    }
    template <class Sink>
    static __device__ __forceinline__ void store(const Ctx& c, const TileGeom&, int, int, const Regs& rg, Smem& sm,
                                                 Sink& sink, int tid) {
        const int j = tid % KT;
#pragma unroll
        for (int i = 0; i < kV; ++i) {
            const int e = tid + i * NT, A = e / KT;
            if (e < 12 * KT) {
                const C2<R> s = rg.v[i];
                sm.v[A][j] = (A >= 6) ? C2<R>{-s.x, s.y} : C2<R>{s.x, -s.y};   // g[at] conj(s)
            }
        }
        __syncthreads();
        if (OPS == 1 || (OPS == 0 && c.nu < 0)) {
#pragma unroll
            for (int i = 0; i < kT; ++i) {
                const int e = tid + i * NT, q = e / KT;
                if (!kFullT && e >= 48 * KT) continue;
#pragma unroll
                for (int at = 0; at < 4; ++at) {
                    C2<R> p = cmul(sm.v[3 * at][j], rg.g[i][0]);
                    p = cfma(p, sm.v[3 * at + 1][j], rg.g[i][1]);
                    p = cfma(p, sm.v[3 * at + 2][j], rg.g[i][2]);
                    sink.put(at * 48 + q, j, p);
                }
            }
            return;
        }
        if constexpr (OPS != 1) {
        // t+[at][d] = 1/2 sum_c v[at][c] U(y)[c][d];  t-[at][d] = 1/2 sum_c v[at][c] conj(U(y-nu)[d][c])
#pragma unroll
        for (int i = 0; i < kV; ++i) {
            const int e = tid + i * NT, q = e / KT;
            if (e >= 12 * KT) continue;
            const int at = q / 3;
            C2<R> tp = {0, 0}, tm = {0, 0};
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                const C2<R> vv = sm.v[3 * at + cc][j];
                tp = cfma(tp, vv, rg.u[i][cc]);
                tm = cadd(tm, cmulc(vv, rg.u[i][3 + cc]));
            }
            sm.tp[q][j] = cscale(tp, (R)0.5);
            sm.tm[q][j] = cscale(tm, (R)0.5);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int e = tid + i * NT, q = e / KT;
            if (!kFullT && e >= 48 * KT) continue;
#pragma unroll
            for (int at = 0; at < 4; ++at) {
                C2<R> p = cmul(sm.tp[3 * at][j], rg.g[i][0]);
                p = cfnma(p, sm.tm[3 * at][j], rg.g[i][3]);
#pragma unroll
                for (int d = 1; d < 3; ++d) {
                    p = cfma(p, sm.tp[3 * at + d][j], rg.g[i][d]);
                    p = cfnma(p, sm.tm[3 * at + d][j], rg.g[i][3 + d]);
                }
                sink.put(at * 48 + q, j, p);
            }
        }
        }
    }
};

template <typename R, int KT, int NT>
using InsertionProducer = InsertionProducerT<R, KT, NT, 0>;
template <typename R, int KT, int NT>
using InsertionLocalProducer = InsertionProducerT<R, KT, NT, 1>;
template <typename R, int KT, int NT>
using InsertionDerivProducer = InsertionProducerT<R, KT, NT, 2>;

}  // namespace c3pt
