// Producers of the factored projection (c3pt_fac.h).  They contract the same
// tensors as the producers of the dense kernels (c3pt_producers.h: Eq. (9)
// meson and nucleon spectators, Eq. (10) insertion) but are split for a
// software pipeline with one workgroup barrier per tile:
//   load_pre(T)   per-site inputs shared by many tasks (noise vector, links,
//                 the G1 block) -> registers Pre
//   stage(T)      Pre -> the tile's LDS buffer Buf (v = gamma-signed noise,
//                 transported noise for the derivative, G1 block)
//   load_main(T)  propagator entries of the thread's tasks -> registers Main
//   contract(T)   Main + Buf -> P slots in LDS
// A tile is KT consecutive sites of one x1 row segment; a thread keeps site
// j = tid % KT.  Sites past the row end load the last site of the segment
// (every load is in bounds and unconditional) and the stage-1 operand of the
// loop is zero there, so they add nothing.
//
// Every producer has 48 task rows r with 48 * KT tasks (r, j) per tile; task
// e = tid + i * NT (i < kT) is thread tid's, and writes the four columns
// col(X, r), X = 0..3.  Slot 16 w + 4 X + loc of P belongs to wave w: the
// 16-column MFMA tile of a wave holds exactly what the wave contracted, so the
// stage-1 GEMM needs no workgroup barrier after the contraction.
#pragma once

#include "c3pt_producers.h"

namespace c3pt {

template <int KT, int NT>
struct FacSlots {
    static constexpr int QW = 64 / KT;        // task rows per wave and i
    static constexpr int RPI = NT / KT;       // task rows per i
    static constexpr int kT = 48 * KT / NT;   // tasks per thread
    static_assert(NT % 64 == 0 && 64 % KT == 0, "a wave holds whole task rows");
    static_assert(48 * KT == kT * NT && QW * kT == 4, "four task rows per wave");
    static __device__ __forceinline__ int slot(int X, int r) {
        const int i = r / RPI, rr = r % RPI;
        return 16 * (rr / QW) + 4 * X + i * QW + rr % QW;
    }
    static __device__ __forceinline__ void of_slot(int s, int& X, int& r) {
        const int w = s >> 4, n = s & 15, loc = n & 3;
        X = n >> 2;
        r = (loc / QW) * RPI + w * QW + loc % QW;
    }
};

// Site of thread tid in a row-segment tile: clamped into the segment.
struct RowSite {
    int n;            // site index x1 + L1 (x2 + L2 x3)
    int x1, x2, x3;
    unsigned np, nm;  // neighbours along the derivative direction (set by its prepare)
};

template <typename R, int KT>
struct FacPut {
    R* P;             // P[slot * PST + 2 * site + re/im]
    int pst;
    __device__ __forceinline__ void put(int slot, int j, C2<R> v) { *(C2<R>*)&P[slot * pst + 2 * j] = v; }
};

// ---------------------------------------------------------------------------
// Meson spectator, Eq. (9): task row r = a'*12 + a*3 + c, X = b'.
// ---------------------------------------------------------------------------
template <typename R, int KT, int NT>
struct FacMesonProd : MesonSpecProducer<R, KT, NT> {
    using Base = MesonSpecProducer<R, KT, NT>;
    using Args = typename Base::Args;
    using Ctx = typename Base::Ctx;
    using S = FacSlots<KT, NT>;
    static constexpr int kP = PerThread<12 * KT, NT>::value;
    static constexpr int kT = S::kT;
    struct Pre { C2<R> v[kP]; };
    struct Main { C2<R> g[kT][3]; };
    struct Buf { C2<R> v[12][KT]; };
    static __device__ __forceinline__ int col(int X, int r) { return X * 48 + r; }
    static __device__ __forceinline__ void prepare(const Ctx&, RowSite&) {}
    static __device__ __forceinline__ void load_pre(const Ctx& c, const TileGeom& tg, const RowSite& rs, Pre& p,
                                                    int tid) {
#pragma unroll
        for (int i = 0; i < kP; ++i) {
            const int e = tid + i * NT;
            if (e < 12 * KT) p.v[i] = c.eta[(unsigned)(e / KT) * (unsigned)tg.V3 + (unsigned)rs.n];
        }
    }
    static __device__ __forceinline__ void stage(const Ctx&, const Pre& p, Buf& b, int tid) {
        const int j = tid % KT;
#pragma unroll
        for (int i = 0; i < kP; ++i) {
            const int e = tid + i * NT, A = e / KT;
            if (e < 12 * KT) b.v[A][j] = (A >= 6) ? C2<R>{-p.v[i].x, -p.v[i].y} : p.v[i];
        }
    }
    static __device__ __forceinline__ void load_main(const Ctx& c, const TileGeom& tg, const RowSite& rs, Main& m,
                                                     int tid) {
        const unsigned V3 = (unsigned)tg.V3, n = (unsigned)rs.n;
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int r = (tid + i * NT) / KT, ap = r / 12, rem = r % 12;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) m.g[i][cc] = c.G[(unsigned)((3 * ap + cc) * 12 + rem) * V3 + n];
        }
    }
    template <class Put>
    static __device__ __forceinline__ void contract(const Ctx&, const Main& m, const Buf& b, Put& out, int tid) {
        const int j = tid % KT;
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int r = (tid + i * NT) / KT, ap = r / 12, al = (r % 12) / 3;
            const R sg = g5<R>(ap) * g5<R>(al);
#pragma unroll
            for (int bp = 0; bp < 4; ++bp) {
                C2<R> p = cmulc(b.v[3 * bp][j], m.g[i][0]);
                p = cadd(p, cmulc(b.v[3 * bp + 1][j], m.g[i][1]));
                p = cadd(p, cmulc(b.v[3 * bp + 2][j], m.g[i][2]));
                out.put(S::slot(bp, r), j, cscale(p, sg));
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Nucleon spectator with epsilon tensors (Eq. (9)): task row r = q * 3 + c'
// with q = a2'*4 + a2, X = b'; column (q*4 + b')*3 + c'.  A task forms the
// column c' of
//   Q[c][c'] = sum eps_{abc} eps_{a'b'c'} G1[(a1',a)][(a1,a')] G2[(a2',b)][(a2,b')]
// (six G2 entries: the two colour columns other than c') and
//   P = g[b'] sum_c eta[(b',c)] Q[c][c'].
// ---------------------------------------------------------------------------
template <typename R, int KT, int NT>
struct FacBaryonProd : BaryonSpecProducer<R, KT, NT> {
    using Base = BaryonSpecProducer<R, KT, NT>;
    using Args = typename Base::Args;
    using Ctx = typename Base::Ctx;
    using S = FacSlots<KT, NT>;
    static constexpr int kP = PerThread<21 * KT, NT>::value;
    static constexpr int kT = S::kT;
    struct Pre { C2<R> v[kP]; };
    struct Main { C2<R> g2[kT][6]; };   // [2x + 0] = G2(x, c'+1), [2x + 1] = G2(x, c'+2) (colours mod 3)
    struct Buf {
        C2<R> v[12][KT];
        C2<R> g1[9][KT];
    };
    static __device__ __forceinline__ int col(int X, int r) { return ((r / 3) * 4 + X) * 3 + r % 3; }
    static __device__ __forceinline__ void prepare(const Ctx&, RowSite&) {}
    static __device__ __forceinline__ void load_pre(const Ctx& c, const TileGeom& tg, const RowSite& rs, Pre& p,
                                                    int tid) {
        const unsigned V3 = (unsigned)tg.V3, n = (unsigned)rs.n;
#pragma unroll
        for (int i = 0; i < kP; ++i) {
            const int e = tid + i * NT, A = e / KT;
            if (e < 21 * KT) {
                // entries 0..11: the noise vector; 12..20: the G1 block of (a1', a1)
                const int cc = A - 12;
                p.v[i] = A < 12 ? c.eta[(unsigned)A * V3 + n]
                                : c.G1[(unsigned)((3 * c.a1p + cc / 3) * 12 + 3 * c.a1 + cc % 3) * V3 + n];
            }
        }
    }
    static __device__ __forceinline__ void stage(const Ctx&, const Pre& p, Buf& b, int tid) {
        const int j = tid % KT;
#pragma unroll
        for (int i = 0; i < kP; ++i) {
            const int e = tid + i * NT, A = e / KT;
            if (e >= 21 * KT) continue;
            if (A < 12) b.v[A][j] = (A >= 6) ? C2<R>{-p.v[i].x, -p.v[i].y} : p.v[i];
            else b.g1[A - 12][j] = p.v[i];
        }
    }
    static __device__ __forceinline__ void load_main(const Ctx& c, const TileGeom& tg, const RowSite& rs, Main& m,
                                                     int tid) {
        const unsigned V3 = (unsigned)tg.V3, n = (unsigned)rs.n;
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int r = (tid + i * NT) / KT, q = r / 3, cp = r % 3;
            const int a2p = q >> 2, a2 = q & 3;
            const int pa = cp == 2 ? 0 : cp + 1, pb = cp == 0 ? 2 : cp - 1;
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                const unsigned row = (unsigned)((3 * a2p + x) * 12 + 3 * a2);
                m.g2[i][2 * x] = c.G2[(row + (unsigned)pa) * V3 + n];
                m.g2[i][2 * x + 1] = c.G2[(row + (unsigned)pb) * V3 + n];
            }
        }
    }
    template <class Put>
    static __device__ __forceinline__ void contract(const Ctx&, const Main& m, const Buf& b, Put& out, int tid) {
        const int j = tid % KT;
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int r = (tid + i * NT) / KT, cp = r % 3;
            const int pa = cp == 2 ? 0 : cp + 1, pb = cp == 0 ? 2 : cp - 1;
            // G1 entries of the colour columns pa, pb for rows 0..2
            C2<R> ga[3], gb[3];
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                ga[x] = b.g1[3 * x + pa][j];
                gb[x] = b.g1[3 * x + pb][j];
            }
            // Q[c] with (a, b) = (c+1, c+2) (+) and (c+2, c+1) (-); primes (pa, pb)
            C2<R> Q[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int ca = (c + 1) % 3, cb = (c + 2) % 3;
                C2<R> t = cmul(ga[ca], m.g2[i][2 * cb + 1]);
                t = cfnma(t, gb[ca], m.g2[i][2 * cb]);
                t = cfnma(t, ga[cb], m.g2[i][2 * ca + 1]);
                Q[c] = cfma(t, gb[cb], m.g2[i][2 * ca]);
            }
#pragma unroll
            for (int bp = 0; bp < 4; ++bp) {
                C2<R> p = cmul(b.v[3 * bp][j], Q[0]);
                p = cfma(p, b.v[3 * bp + 1][j], Q[1]);
                p = cfma(p, b.v[3 * bp + 2][j], Q[2]);
                out.put(S::slot(bp, r), j, p);
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Insertion, Eq. (10), local operator: task row r = bt*12 + b*3 + c, X = at.
// ---------------------------------------------------------------------------
template <typename R, int KT, int NT>
struct FacInsLocalProd : InsertionProducerT<R, KT, NT, 1> {
    using Base = InsertionProducerT<R, KT, NT, 1>;
    using Args = typename Base::Args;
    using Ctx = typename Base::Ctx;
    using S = FacSlots<KT, NT>;
    static constexpr int kP = PerThread<12 * KT, NT>::value;
    static constexpr int kT = S::kT;
    struct Pre { C2<R> s[kP]; };
    struct Main { C2<R> g[kT][3]; };
    struct Buf { C2<R> v[12][KT]; };
    static __device__ __forceinline__ int col(int X, int r) { return X * 48 + r; }
    static __device__ __forceinline__ void prepare(const Ctx&, RowSite&) {}
    static __device__ __forceinline__ void load_pre(const Ctx& c, const TileGeom& tg, const RowSite& rs, Pre& p,
                                                    int tid) {
#pragma unroll
        for (int i = 0; i < kP; ++i) {
            const int e = tid + i * NT;
            if (e < 12 * KT) p.s[i] = c.s[(unsigned)(e / KT) * (unsigned)tg.V3 + (unsigned)rs.n];
        }
    }
    static __device__ __forceinline__ void stage(const Ctx&, const Pre& p, Buf& b, int tid) {
        const int j = tid % KT;
#pragma unroll
        for (int i = 0; i < kP; ++i) {
            const int e = tid + i * NT, A = e / KT;
            if (e < 12 * KT) {
                const C2<R> s = p.s[i];
                b.v[A][j] = (A >= 6) ? C2<R>{-s.x, s.y} : C2<R>{s.x, -s.y};   // g[at] conj(s)
            }
        }
    }
    static __device__ __forceinline__ void load_main(const Ctx& c, const TileGeom& tg, const RowSite& rs, Main& m,
                                                     int tid) {
        const unsigned V3 = (unsigned)tg.V3, n = (unsigned)rs.n;
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int r = (tid + i * NT) / KT, bt = r / 12, rem = r % 12;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) m.g[i][cc] = c.Gf[(unsigned)((3 * bt + cc) * 12 + rem) * V3 + n];
        }
    }
    template <class Put>
    static __device__ __forceinline__ void contract(const Ctx&, const Main& m, const Buf& b, Put& out, int tid) {
        const int j = tid % KT;
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int r = (tid + i * NT) / KT;
#pragma unroll
            for (int at = 0; at < 4; ++at) {
                C2<R> p = cmul(b.v[3 * at][j], m.g[i][0]);
                p = cfma(p, b.v[3 * at + 1][j], m.g[i][1]);
                p = cfma(p, b.v[3 * at + 2][j], m.g[i][2]);
                out.put(S::slot(at, r), j, p);
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Insertion, Eq. (10), the four covariant derivatives gamma_mu D_nu: the
// derivative acts on the stochastic vector (transport task (at, d) per site),
//   t+[at][d] = 1/2 sum_c v[at][c] U_nu(y)[c][d],
//   t-[at][d] = 1/2 sum_c v[at][c] conj(U_nu(y - nu)[d][c]),
//   P = sum_d t+[at][d] G(y + nu)[(bt,d)][(b,c)] - t-[at][d] G(y - nu)[(bt,d)][(b,c)].
// Task row r = bt*12 + b*3 + c, X = at.
// ---------------------------------------------------------------------------
template <typename R, int KT, int NT>
struct FacInsDerivProd : InsertionProducerT<R, KT, NT, 2> {
    using Base = InsertionProducerT<R, KT, NT, 2>;
    using Args = typename Base::Args;
    // the base context plus the stride, extent and wrap (stride x extent) of
    // direction nu in the site index (stride 0 for the time direction)
    struct Ctx : Base::Ctx {
        int st, ext, wrap;
    };
    static __device__ __forceinline__ Ctx with_dir(const typename Base::Ctx& b, const int (&L)[3]) {
        Ctx c;
        static_cast<typename Base::Ctx&>(c) = b;
        // sums of products with direction flags: a select chain on nu would
        // become a lookup table in memory
        const int f0 = c.nu == 0, f1 = c.nu == 1, f2 = c.nu == 2;
        c.st = f0 + f1 * L[0] + f2 * L[0] * L[1];
        c.ext = f0 * L[0] + f1 * L[1] + (1 - f0 - f1) * L[2];
        c.wrap = c.st * c.ext;
        return c;
    }
    static __device__ __forceinline__ Ctx resolve(const Args& a, int V3, int cb) {
        return with_dir(Base::resolve(a, V3, cb), a.L);
    }
    static __device__ __forceinline__ Ctx resolve(const BatchJob& b, int V3, int cb) {
        return with_dir(Base::resolve(b, V3, cb), b.L);
    }
    using S = FacSlots<KT, NT>;
    static constexpr int kP = PerThread<12 * KT, NT>::value;
    static constexpr int kT = S::kT;
    struct Pre {
        C2<R> s[kP][3];   // s[(at, c)], c = 0..2, of transport task (at, d)
        C2<R> u[kP][6];   // U(y)[c][d], then U(y - nu)[d][c]
    };
    struct Main { C2<R> g[kT][6]; };   // G(y + nu)[(bt, d)][(b, c)], d = 0..2, then G(y - nu)
    struct Buf {
        C2<R> tp[12][KT];
        C2<R> tm[12][KT];
    };
    static __device__ __forceinline__ int col(int X, int r) { return X * 48 + r; }
    // neighbour sites y +- nu of the thread's site, once per tile (periodic;
    // the time direction reads the adjacent slices at y itself)
    static __device__ __forceinline__ void prepare(const Ctx& c, RowSite& rs) {
        const int f0 = c.nu == 0, f1 = c.nu == 1;
        const int x = f0 * rs.x1 + f1 * rs.x2 + (1 - f0 - f1) * rs.x3;
        rs.np = (unsigned)(rs.n + c.st - (x == c.ext - 1 ? c.wrap : 0));
        rs.nm = (unsigned)(rs.n - c.st + (x == 0 ? c.wrap : 0));
    }
    static __device__ __forceinline__ void load_pre(const Ctx& c, const TileGeom& tg, const RowSite& rs, Pre& p,
                                                    int tid) {
        const unsigned V3 = (unsigned)tg.V3, n = (unsigned)rs.n, nm = rs.nm;
#pragma unroll
        for (int i = 0; i < kP; ++i) {
            const int e = tid + i * NT, q = e / KT, at = q / 3, d = q % 3;
            if (e < 12 * KT) {
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    p.s[i][cc] = c.s[(unsigned)(3 * at + cc) * V3 + n];
                    p.u[i][cc] = c.U[(unsigned)(cc * 3 + d) * V3 + n];
                    p.u[i][3 + cc] = c.Um[(unsigned)(d * 3 + cc) * V3 + nm];
                }
            }
        }
    }
    static __device__ __forceinline__ void stage(const Ctx&, const Pre& p, Buf& b, int tid) {
        const int j = tid % KT;
#pragma unroll
        for (int i = 0; i < kP; ++i) {
            const int e = tid + i * NT, q = e / KT, at = q / 3;
            if (e >= 12 * KT) continue;
            C2<R> tp = {0, 0}, tm = {0, 0};
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                const C2<R> s = p.s[i][cc];
                const C2<R> v = (at >= 2) ? C2<R>{-s.x, s.y} : C2<R>{s.x, -s.y};   // g[at] conj(s)
                tp = cfma(tp, v, p.u[i][cc]);
                tm = cadd(tm, cmulc(v, p.u[i][3 + cc]));
            }
            b.tp[q][j] = cscale(tp, (R)0.5);
            b.tm[q][j] = cscale(tm, (R)0.5);
        }
    }
    static __device__ __forceinline__ void load_main(const Ctx& c, const TileGeom& tg, const RowSite& rs, Main& m,
                                                     int tid) {
        const unsigned V3 = (unsigned)tg.V3, np = rs.np, nm = rs.nm;
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int r = (tid + i * NT) / KT, bt = r / 12, rem = r % 12;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const unsigned plane = (unsigned)((3 * bt + d) * 12 + rem) * V3;
                m.g[i][d] = c.Gf[plane + np];
                m.g[i][3 + d] = c.Gb[plane + nm];
            }
        }
    }
    // the contraction of spins at in [X0, X1): a wave may issue loads between
    // two parts
    static constexpr bool kSplitContract = true;
    template <int X0, int X1, class Put>
    static __device__ __forceinline__ void contract_part(const Ctx&, const Main& m, const Buf& b, Put& out,
                                                         int tid) {
        const int j = tid % KT;
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int r = (tid + i * NT) / KT;
#pragma unroll
            for (int at = X0; at < X1; ++at) {
                C2<R> p = cmul(b.tp[3 * at][j], m.g[i][0]);
                p = cfnma(p, b.tm[3 * at][j], m.g[i][3]);
#pragma unroll
                for (int d = 1; d < 3; ++d) {
                    p = cfma(p, b.tp[3 * at + d][j], m.g[i][d]);
                    p = cfnma(p, b.tm[3 * at + d][j], m.g[i][3 + d]);
                }
                out.put(S::slot(at, r), j, p);
            }
        }
    }
    template <class Put>
    static __device__ __forceinline__ void contract(const Ctx& c, const Main& m, const Buf& b, Put& out, int tid) {
        contract_part<0, 4>(c, m, b, out, tid);
    }
};

}  // namespace c3pt
