// Left derivative of the symmetrized insertion <->D_nu = 1/2 (->D_nu - <-D_nu)
// for the factored projection (c3pt_fac.h).
//
// <-D_nu acts on the insertion's antiquark field.  In the factorized insertion
// part (Eq. (10)) that field is the conjugated gamma5 s, and the lattice left
// derivative psibar(y) <-D_nu = 1/2 [psibar(y+nu) U_nu(y)^dag - psibar(y-nu) U_nu(y-nu)]
// becomes the ordinary covariant derivative of the colour vector s:
//   (D_nu s)[at][c] = 1/2 sum_d U_nu(y)[c][d] s(y+nu)[at][d] - conj(U_nu(y-nu)[d][c]) s(y-nu)[at][d],
// after which the contraction is the local one with G(y):
//   P = sum_c v[at][c] G(y)[(bt,c)][(b,c_src)],  v = g[at] conj(D_nu s).
// Transport task (at, c) per site; the time direction reads s on the
// neighbouring timeslices at the same site.
#pragma once

#include "c3pt_fac_prod.h"

namespace c3pt {

struct InsertionLeftArgs : InsertionArgs {
    const void* sn[kMaxTauPerLaunch];   // s(tau + 1) [N][12][V3]
    const void* sp[kMaxTauPerLaunch];   // s(tau - 1)
};

// Column blocks of an n_ops = 9 insertion: op = 5 + nu.
template <typename R, int KT, int NT>
struct FacInsLeftProd {
    using Args = InsertionLeftArgs;
    using S = FacSlots<KT, NT>;
    static constexpr int kP = PerThread<12 * KT, NT>::value;
    static constexpr int kT = S::kT;
    struct Ctx {
        const C2<R>* G;    // G(y) on tau
        const C2<R>* sf;   // s read at y + nu (time: slice tau + 1)
        const C2<R>* sb;   // s read at y - nu (time: slice tau - 1)
        const C2<R>* U;    // U_nu(y)
        const C2<R>* Um;   // U_nu(y - nu) (time: slice tau - 1)
        int nu;
        int st, ext, wrap; // stride, extent and stride x extent of nu in the site index (time: 0, L3, 0)
    };
    struct Pre {
        C2<R> sf[kP][3];   // s(y + nu)[at][d], d = 0..2, of transport task (at, c)
        C2<R> sb[kP][3];   // s(y - nu)[at][d]
        C2<R> u[kP][6];    // U(y)[c][d], then U(y - nu)[d][c]
    };
    struct Main { C2<R> g[kT][3]; };   // G(y)[(bt, c)][(b, c_src)], c = 0..2
    struct Buf { C2<R> v[12][KT]; };
    static __device__ __forceinline__ int col(int X, int r) { return X * 48 + r; }
    static __device__ __forceinline__ int colblock(const Args& a, int share, int within) {
        const int noise = within / a.op_cnt, op = a.op_lo + within % a.op_cnt;
        return (noise * a.n_tau + share) * a.n_ops + op;
    }
    static __device__ __forceinline__ Ctx resolve(const Args& a, int V3, int cb) {
        const int op = cb % a.n_ops, rest = cb / a.n_ops;
        const int tl = rest % a.n_tau, noise = rest / a.n_tau;
        Ctx c;
        c.nu = op - 5;
        const int f0 = c.nu == 0, f1 = c.nu == 1, f2 = c.nu == 2;
        const bool time = c.nu == 3;
        const size_t off = (size_t)noise * 12 * V3;
        c.G = (const C2<R>*)a.G[tl];
        c.sf = (const C2<R>*)(time ? a.sn[tl] : a.s[tl]) + off;
        c.sb = (const C2<R>*)(time ? a.sp[tl] : a.s[tl]) + off;
        c.U = (const C2<R>*)a.U[tl] + (size_t)c.nu * 9 * V3;
        c.Um = time ? (const C2<R>*)a.Up[tl] + (size_t)27 * V3 : c.U;
        c.st = f0 + f1 * a.L[0] + f2 * a.L[0] * a.L[1];
        c.ext = f0 * a.L[0] + f1 * a.L[1] + (1 - f0 - f1) * a.L[2];
        c.wrap = c.st * c.ext;
        return c;
    }
    static __device__ __forceinline__ void prepare(const Ctx& c, RowSite& rs) {
        const int f0 = c.nu == 0, f1 = c.nu == 1;
        const int x = f0 * rs.x1 + f1 * rs.x2 + (1 - f0 - f1) * rs.x3;
        rs.np = (unsigned)(rs.n + c.st - (x == c.ext - 1 ? c.wrap : 0));
        rs.nm = (unsigned)(rs.n - c.st + (x == 0 ? c.wrap : 0));
    }
    static __device__ __forceinline__ void load_pre(const Ctx& c, const TileGeom& tg, const RowSite& rs, Pre& p,
                                                    int tid) {
        const unsigned V3 = (unsigned)tg.V3, n = (unsigned)rs.n, np = rs.np, nm = rs.nm;
#pragma unroll
        for (int i = 0; i < kP; ++i) {
            const int e = tid + i * NT, q = e / KT, at = q / 3, cc = q % 3;
            if (e < 12 * KT) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    p.sf[i][d] = c.sf[(unsigned)(3 * at + d) * V3 + np];
                    p.sb[i][d] = c.sb[(unsigned)(3 * at + d) * V3 + nm];
                    p.u[i][d] = c.U[(unsigned)(cc * 3 + d) * V3 + n];
                    p.u[i][3 + d] = c.Um[(unsigned)(d * 3 + cc) * V3 + nm];
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
            C2<R> ds = {0, 0};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                ds = cfma(ds, p.u[i][d], p.sf[i][d]);
                ds = csub(ds, cmulc(p.sb[i][d], p.u[i][3 + d]));
            }
            ds = cscale(ds, (R)0.5);
            b.v[q][j] = (at >= 2) ? C2<R>{-ds.x, ds.y} : C2<R>{ds.x, -ds.y};   // g[at] conj(D s)
        }
    }
    static __device__ __forceinline__ void load_main(const Ctx& c, const TileGeom& tg, const RowSite& rs, Main& m,
                                                     int tid) {
        const unsigned V3 = (unsigned)tg.V3, n = (unsigned)rs.n;
#pragma unroll
        for (int i = 0; i < kT; ++i) {
            const int r = (tid + i * NT) / KT, bt = r / 12, rem = r % 12;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) m.g[i][cc] = c.G[(unsigned)((3 * bt + cc) * 12 + rem) * V3 + n];
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

}  // namespace c3pt
