// Kernels of libc3pt for gfx950 (MI355X).
//
// Fused contraction + momentum projection.  One workgroup owns one column
// block (192 spin-colour components of one noise vector / timeslice / operator)
// and one chunk of spatial sites.  For every tile of KT sites it
//   1. builds the phases exp(sigma 2 pi i k.(x-r)/L) of the tile in LDS from
//      per-direction root-of-unity tables (integer phase index, exact),
//   2. contracts the propagator with the noise / stochastic vector for the
//      tile into an LDS tile P[col][site] (the "producer": Eq. (9) spectator,
//      Eq. (10) insertion with optional covariant derivative, or the
//      epsilon-tensor baryon spectator),
//   3. multiplies phases x P with MFMA 16x16x4 (FP32 or FP64), the complex
//      product written as a real GEMM whose A rows interleave (re, im) of each
//      momentum and whose K runs over (site, re/im).
// FP32 accumulators never span more than kMaxSitesPerChunkF32 sites; each
// workgroup writes its chunk's sums in FP64 and a separate kernel reduces the
// chunks in a fixed order (deterministic, no floating-point atomics).
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
template <typename R>
__device__ __forceinline__ C2<R> cconj(C2<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ C2<R> cscale(C2<R> a, R s) { return {a.x * s, a.y * s}; }

// Accumulator layout of the 16x16x4 MFMAs on gfx950 (lane l, register j):
//   FP32: D[4*(l/16) + j][l%16]        FP64: D[4*j + l/16][l%16]
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

// v mod L for 0 <= v < 2^20 using a float reciprocal and one correction step.
__device__ __forceinline__ int mod_small(int v, int L, float invL) {
    int q = (int)((float)v * invL);
    int r = v - q * L;
    r += (r < 0) ? L : 0;
    r -= (r >= L) ? L : 0;
    return r;
}

// gamma5 = diag(1, 1, -1, -1) in the DeGrand-Rossi basis: sign of spin s.
__device__ __forceinline__ float g5f(int s) { return s < 2 ? 1.0f : -1.0f; }

// ---------------------------------------------------------------------------
// Producers: fill P[col][site] (LDS, interleaved re/im, column stride PST) for
// one site tile.  Sites j >= nsite are written as zero.
// ---------------------------------------------------------------------------
struct TileGeom {
    int V3, L1, L2, L3;
};

// Meson spectator, Eq. (9):
//   P[(b',a',a,c)] = g[b'] g[a'] g[a] sum_c' eta[(b',c')] conj(G[(a',c')][(a,c)])
template <typename R, int KT, int NT>
struct MesonSpecProducer {
    using Args = MesonSpecArgs;
    struct Smem {
        C2<R> v[12][KT];
    };
    template <int PST>
    static __device__ __forceinline__ void produce(const Args& a, const TileGeom& tg, int cb, int t0,
                                                   int nsite, R* sP, Smem& sm, int tid) {
        const size_t V3 = (size_t)tg.V3;
        const C2<R>* G = (const C2<R>*)a.G;
        const C2<R>* eta = (const C2<R>*)a.eta + (size_t)cb * 12 * V3;
        for (int e = tid; e < 12 * KT; e += NT) {
            const int A = e / KT, j = e % KT;
            C2<R> v = {0, 0};
            if (j < nsite) {
                v = eta[(size_t)A * V3 + t0 + j];
                if (A >= 6) v = {-v.x, -v.y};
            }
            sm.v[A][j] = v;
        }
        __syncthreads();
        for (int e = tid; e < 48 * KT; e += NT) {
            const int j = e % KT, q = e / KT;          // q = a'*12 + a*3 + c
            const int ap = q / 12, rem = q % 12, al = rem / 3;
            C2<R> g[3] = {{0, 0}, {0, 0}, {0, 0}};
            if (j < nsite) {
                const size_t n = (size_t)t0 + j;
#pragma unroll
                for (int c = 0; c < 3; ++c) g[c] = G[(size_t)((3 * ap + c) * 12 + rem) * V3 + n];
            }
            const R sg = (R)(g5f(ap) * g5f(al));
#pragma unroll
            for (int bp = 0; bp < 4; ++bp) {
                C2<R> p = {0, 0};
#pragma unroll
                for (int c = 0; c < 3; ++c) p = cadd(p, cmulc(sm.v[3 * bp + c][j], g[c]));
                const int col = bp * 48 + q;
                sP[col * PST + 2 * j] = p.x * sg;
                sP[col * PST + 2 * j + 1] = p.y * sg;
            }
        }
    }
};

// Nucleon-type spectator with epsilon tensors at sink and source.  Column
// block cb = noise * 16 + (a1' * 4 + a1); columns (a2', a2, b', c').
//   P = g[b'] sum_c eta[(b',c)] Q[c][c'],
//   Q[c][c'] = sum eps_{abc} eps_{a'b'c'} G1[(a1',a)][(a1,a')] G2[(a2',b)][(a2,b')]
template <typename R, int KT, int NT>
struct BaryonSpecProducer {
    using Args = BaryonSpecArgs;
    struct Smem {
        C2<R> v[12][KT];
        C2<R> g1[9][KT];
    };
    template <int PST>
    static __device__ __forceinline__ void produce(const Args& a, const TileGeom& tg, int cb, int t0,
                                                   int nsite, R* sP, Smem& sm, int tid) {
        const size_t V3 = (size_t)tg.V3;
        const int noise = cb >> 4, blk = cb & 15;
        const int a1p = blk >> 2, a1 = blk & 3;
        const C2<R>* G1 = (const C2<R>*)a.G1;
        const C2<R>* G2 = (const C2<R>*)a.G2;
        const C2<R>* eta = (const C2<R>*)a.eta + (size_t)noise * 12 * V3;
        for (int e = tid; e < 21 * KT; e += NT) {
            const int A = e / KT, j = e % KT;
            C2<R> v = {0, 0};
            if (A < 12) {
                if (j < nsite) {
                    v = eta[(size_t)A * V3 + t0 + j];
                    if (A >= 6) v = {-v.x, -v.y};
                }
                sm.v[A][j] = v;
            } else {
                const int cc = A - 12, ca = cc / 3, cap = cc % 3;
                if (j < nsite) v = G1[(size_t)((3 * a1p + ca) * 12 + 3 * a1 + cap) * V3 + t0 + j];
                sm.g1[cc][j] = v;
            }
        }
        __syncthreads();
        for (int e = tid; e < 16 * KT; e += NT) {
            const int j = e % KT, q = e / KT;   // q = a2' * 4 + a2
            const int a2p = q >> 2, a2 = q & 3;
            C2<R> g2[9];
#pragma unroll
            for (int cc = 0; cc < 9; ++cc) {
                g2[cc] = {0, 0};
                if (j < nsite)
                    g2[cc] = G2[(size_t)((3 * a2p + cc / 3) * 12 + 3 * a2 + cc % 3) * V3 + t0 + j];
            }
            C2<R> g1[9];
#pragma unroll
            for (int cc = 0; cc < 9; ++cc) g1[cc] = sm.g1[cc][j];
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
                    t = cadd(t, cmul(g1[cb2 * 3 + pb], g2[ca * 3 + pa]));
                    Q[c * 3 + cp] = t;
                }
            }
#pragma unroll
            for (int bp = 0; bp < 4; ++bp) {
                const C2<R> v0 = sm.v[3 * bp][j], v1 = sm.v[3 * bp + 1][j], v2 = sm.v[3 * bp + 2][j];
#pragma unroll
                for (int cp = 0; cp < 3; ++cp) {
                    C2<R> p = cmul(v0, Q[cp]);
                    p = cadd(p, cmul(v1, Q[3 + cp]));
                    p = cadd(p, cmul(v2, Q[6 + cp]));
                    const int col = (q * 4 + bp) * 3 + cp;
                    sP[col * PST + 2 * j] = p.x;
                    sP[col * PST + 2 * j + 1] = p.y;
                }
            }
        }
    }
};

// Insertion, Eq. (10).  Column block cb = ((noise * n_tau) + tau) * n_ops + op;
// columns (at, bt, b, c).  op 0: P = sum_c' v[at][c'] G[(bt,c')][(b,c)] with
// v = g[at] conj(s[(at,c')]).  op 1+nu: the covariant derivative is moved onto
// the stochastic vector, t+ = 1/2 v U_nu(y), t- = 1/2 v U_nu(y-nu)^dag, and
// P = sum_d t+[at][d] G(y+nu)[(bt,d)][(b,c)] - t-[at][d] G(y-nu)[(bt,d)][(b,c)].
template <typename R, int KT, int NT>
struct InsertionProducer {
    using Args = InsertionArgs;
    struct Smem {
        C2<R> v[12][KT];
        C2<R> tp[12][KT];
        C2<R> tm[12][KT];
        int nb[2][KT];
    };
    template <int PST>
    static __device__ __forceinline__ void produce(const Args& a, const TileGeom& tg, int cb, int t0,
                                                   int nsite, R* sP, Smem& sm, int tid) {
        const size_t V3 = (size_t)tg.V3;
        const int op = cb % a.n_ops;
        const int rest = cb / a.n_ops;
        const int tl = rest % a.n_tau;
        const int noise = rest / a.n_tau;
        const C2<R>* s = (const C2<R>*)a.s[tl] + (size_t)noise * 12 * V3;
        for (int e = tid; e < 12 * KT; e += NT) {
            const int A = e / KT, j = e % KT;
            C2<R> v = {0, 0};
            if (j < nsite) {
                v = s[(size_t)A * V3 + t0 + j];
                v = (A >= 6) ? C2<R>{-v.x, v.y} : C2<R>{v.x, -v.y};   // g[at] conj(s)
            }
            sm.v[A][j] = v;
        }
        if (op == 0) {
            __syncthreads();
            const C2<R>* G = (const C2<R>*)a.G[tl];
            for (int e = tid; e < 48 * KT; e += NT) {
                const int j = e % KT, q = e / KT;   // q = bt*12 + b*3 + c
                const int bt = q / 12, rem = q % 12;
                C2<R> g[3] = {{0, 0}, {0, 0}, {0, 0}};
                if (j < nsite) {
                    const size_t n = (size_t)t0 + j;
#pragma unroll
                    for (int c = 0; c < 3; ++c) g[c] = G[(size_t)((3 * bt + c) * 12 + rem) * V3 + n];
                }
#pragma unroll
                for (int at = 0; at < 4; ++at) {
                    C2<R> p = cmul(sm.v[3 * at][j], g[0]);
                    p = cadd(p, cmul(sm.v[3 * at + 1][j], g[1]));
                    p = cadd(p, cmul(sm.v[3 * at + 2][j], g[2]));
                    const int col = at * 48 + q;
                    sP[col * PST + 2 * j] = p.x;
                    sP[col * PST + 2 * j + 1] = p.y;
                }
            }
            return;
        }
        const int nu = op - 1;
        // neighbour site indices (spatial directions); time: same site, other slice
        if (tid < KT) {
            const int j = tid;
            int np = 0, nm = 0;
            if (j < nsite) {
                const int n = t0 + j;
                const int x1 = n % tg.L1, x2 = (n / tg.L1) % tg.L2, x3 = n / (tg.L1 * tg.L2);
                if (nu == 0) {
                    const int xp = (x1 + 1 == tg.L1) ? 0 : x1 + 1, xm = (x1 == 0) ? tg.L1 - 1 : x1 - 1;
                    np = xp + tg.L1 * (x2 + tg.L2 * x3);
                    nm = xm + tg.L1 * (x2 + tg.L2 * x3);
                } else if (nu == 1) {
                    const int xp = (x2 + 1 == tg.L2) ? 0 : x2 + 1, xm = (x2 == 0) ? tg.L2 - 1 : x2 - 1;
                    np = x1 + tg.L1 * (xp + tg.L2 * x3);
                    nm = x1 + tg.L1 * (xm + tg.L2 * x3);
                } else if (nu == 2) {
                    const int xp = (x3 + 1 == tg.L3) ? 0 : x3 + 1, xm = (x3 == 0) ? tg.L3 - 1 : x3 - 1;
                    np = x1 + tg.L1 * (x2 + tg.L2 * xp);
                    nm = x1 + tg.L1 * (x2 + tg.L2 * xm);
                } else {
                    np = n;
                    nm = n;
                }
            }
            sm.nb[0][j] = np;
            sm.nb[1][j] = nm;
        }
        __syncthreads();
        // transports t+[at][d] = 1/2 sum_c v[at][c] U(y)[c][d];
        //            t-[at][d] = 1/2 sum_c v[at][c] conj(U(y-nu)[d][c])
        {
            const C2<R>* U = (const C2<R>*)a.U[tl] + (size_t)nu * 9 * V3;
            const C2<R>* Um = (nu < 3) ? U : (const C2<R>*)a.Up[tl] + (size_t)3 * 9 * V3;
            for (int e = tid; e < 12 * KT; e += NT) {
                const int j = e % KT, q = e / KT;   // q = at*3 + d
                const int at = q / 3, d = q % 3;
                C2<R> tp = {0, 0}, tm = {0, 0};
                if (j < nsite) {
                    const size_t n = (size_t)t0 + j;
                    const size_t nmi = (size_t)sm.nb[1][j];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const C2<R> vv = sm.v[3 * at + c][j];
                        tp = cadd(tp, cmul(vv, U[(size_t)(c * 3 + d) * V3 + n]));
                        tm = cadd(tm, cmulc(vv, Um[(size_t)(d * 3 + c) * V3 + nmi]));
                    }
                }
                sm.tp[q][j] = cscale(tp, (R)0.5);
                sm.tm[q][j] = cscale(tm, (R)0.5);
            }
        }
        __syncthreads();
        const C2<R>* Gf = (const C2<R>*)((nu < 3) ? a.G[tl] : a.Gn[tl]);
        const C2<R>* Gb = (const C2<R>*)((nu < 3) ? a.G[tl] : a.Gp[tl]);
        for (int e = tid; e < 48 * KT; e += NT) {
            const int j = e % KT, q = e / KT;
            const int bt = q / 12, rem = q % 12;
            C2<R> gp[3] = {{0, 0}, {0, 0}, {0, 0}}, gm[3] = {{0, 0}, {0, 0}, {0, 0}};
            if (j < nsite) {
                const size_t np = (size_t)sm.nb[0][j], nm = (size_t)sm.nb[1][j];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    gp[d] = Gf[(size_t)((3 * bt + d) * 12 + rem) * V3 + np];
                    gm[d] = Gb[(size_t)((3 * bt + d) * 12 + rem) * V3 + nm];
                }
            }
#pragma unroll
            for (int at = 0; at < 4; ++at) {
                C2<R> p = {0, 0};
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    p = cadd(p, cmul(sm.tp[3 * at + d][j], gp[d]));
                    p = csub(p, cmul(sm.tm[3 * at + d][j], gm[d]));
                }
                const int col = at * 48 + q;
                sP[col * PST + 2 * j] = p.x;
                sP[col * PST + 2 * j + 1] = p.y;
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Fused contraction + projection kernel.
// ---------------------------------------------------------------------------
template <typename R, int KT, int MTMAX, int WM, int WN, int CT, template <typename, int, int> class ProdT>
__global__ void __launch_bounds__(64 * WM * WN)
proj_kernel(ProjGrid pg, typename ProdT<R, KT, 64 * WM * WN>::Args pa) {
    constexpr int NT = 64 * WM * WN;
    using Prod = ProdT<R, KT, NT>;
    using MF = Mfma<R>;
    using acc_t = typename MF::acc_t;
    constexpr int PST = 2 * KT + 4;       // padded column stride of the P tile
    constexpr int MROWS = 8 * MTMAX;
    constexpr int RT_PER_WAVE = MTMAX / WM;
    static_assert(WN * CT * 16 == kBlockCols, "column block must be 192 wide");
    static_assert(MTMAX % WM == 0, "row tiles must split evenly over waves");
    static_assert(KT % 2 == 0, "site tile must hold whole K steps");

    __shared__ R sP[kBlockCols * PST];
    __shared__ C2<R> sPh[KT * MROWS];
    __shared__ C2<R> sTab[3 * kMaxL];
    __shared__ int sXr[3][KT];
    __shared__ typename Prod::Smem psm;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wn = wave % WN, wm = wave / WN;
    const int cb = blockIdx.x, chunk = blockIdx.y;
    const PhaseSpec& ph = pg.ph;
    const int L1 = ph.L[0], L2 = ph.L[1], L3 = ph.L[2];
    const int n_mom = ph.n_mom;
    const int mt = (n_mom + 7) >> 3;
    const TileGeom tg = {pg.V3, L1, L2, L3};

    // Root-of-unity tables exp(sigma 2 pi i n / L_j), n < L_j, per direction.
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
    const float inv1 = 1.0f / (float)L1, inv2 = 1.0f / (float)L2, inv3 = 1.0f / (float)L3;

    acc_t acc[RT_PER_WAVE][CT];
#pragma unroll
    for (int i = 0; i < RT_PER_WAVE; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    // A-operand rows: row r = lane & 15 of a 16-row tile holds (momentum
    // 8*rt + m_off, part), part 0 = real row, 1 = imaginary row, arranged so that
    // accumulator registers (0,1) / (2,3) of lane l are (re, im) of momenta
    // 8*rt + 2*(l/16) and 8*rt + 2*(l/16) + 1 for both accumulator layouts.
    // K index lane>>4 -> site (lane>>5), component (lane>>4)&1 of P.
    // Real row: (phi_re, -phi_im); imaginary row: (phi_im, phi_re).
    const int arow = lane & 15;
    const int part = MF::kRowsByRegister ? ((arow >> 2) & 1) : (arow & 1);
    const int a_moff = MF::kRowsByRegister ? (2 * (arow & 3) + (arow >> 3)) : (arow >> 1);
    const int comp = (lane >> 4) & 1;
    const bool take_re = (part == comp);
    const bool negate = (part == 0) && (comp == 1);
    const int a_site = lane >> 5;

    const int s_lo = chunk * pg.chunk_sites;
    const int s_hi = min(pg.V3, s_lo + pg.chunk_sites);
    for (int t0 = s_lo; t0 < s_hi; t0 += KT) {
        const int nsite = min(KT, s_hi - t0);
        __syncthreads();
        if (tid < KT) {
            const int n = t0 + tid;
            const int x1 = n % L1, x2 = (n / L1) % L2, x3 = n / (L1 * L2);
            int d1 = x1 - ph.r[0], d2 = x2 - ph.r[1], d3 = x3 - ph.r[2];
            d1 += (d1 < 0) ? L1 : 0;
            d2 += (d2 < 0) ? L2 : 0;
            d3 += (d3 < 0) ? L3 : 0;
            sXr[0][tid] = d1;
            sXr[1][tid] = d2;
            sXr[2][tid] = d3;
        }
        __syncthreads();
        for (int e = tid; e < KT * MROWS; e += NT) {
            const int j = e / MROWS, m = e % MROWS;
            C2<R> v = {0, 0};
            if (j < nsite && m < n_mom) {
                const int i1 = (int)ph.k[0][m] * sXr[0][j];
                const int i2 = (int)ph.k[1][m] * sXr[1][j];
                const int i3 = (int)ph.k[2][m] * sXr[2][j];
                if (ph.cubic) {
                    v = sTab[mod_small(i1 + i2 + i3, L1, inv1)];
                } else {
                    v = cmul(cmul(sTab[mod_small(i1, L1, inv1)], sTab[L1 + mod_small(i2, L2, inv2)]),
                             sTab[L1 + L2 + mod_small(i3, L3, inv3)]);
                }
            }
            sPh[j * MROWS + m] = v;
        }
        Prod::template produce<PST>(pa, tg, cb, t0, nsite, sP, psm, tid);
        __syncthreads();
#pragma unroll 2
        for (int ks = 0; ks < KT / 2; ++ks) {
            R b[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int col = 16 * (wn * CT + ct) + (lane & 15);
                b[ct] = sP[col * PST + 4 * ks + (lane >> 4)];
            }
#pragma unroll
            for (int rt = 0; rt < RT_PER_WAVE; ++rt) {
                const int rtg = wm * RT_PER_WAVE + rt;
                if (rtg < mt) {
                    const C2<R> p = sPh[(2 * ks + a_site) * MROWS + 8 * rtg + a_moff];
                    R av = take_re ? p.x : p.y;
                    av = negate ? -av : av;
#pragma unroll
                    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = MF::mac(av, b[ct], acc[rt][ct]);
                }
            }
        }
    }

    // FP64 partial sums of this chunk: partial[chunk][cb][m][col].
    const size_t base = ((size_t)chunk * pg.n_colblocks + cb) * (size_t)n_mom;
#pragma unroll
    for (int rt = 0; rt < RT_PER_WAVE; ++rt) {
        const int rtg = wm * RT_PER_WAVE + rt;
        if (rtg >= mt) continue;
        const int m0 = 8 * rtg + 2 * (lane >> 4);
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const int col = 16 * (wn * CT + ct) + (lane & 15);
            if (m0 < n_mom)
                pg.partial[(base + m0) * kBlockCols + col] =
                    make_double2((double)acc[rt][ct][0], (double)acc[rt][ct][1]);
            if (m0 + 1 < n_mom)
                pg.partial[(base + m0 + 1) * kBlockCols + col] =
                    make_double2((double)acc[rt][ct][2], (double)acc[rt][ct][3]);
        }
    }
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reduction of the split-site partial sums.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) reduce_kernel(ReduceArgs a) {
    const size_t total = (size_t)a.n_groups * a.n_mom_grp * a.group_cols;
    const int blocks_per_group = a.group_cols / kBlockCols;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(idx % a.group_cols);
        const size_t rest = idx / a.group_cols;
        const int m = (int)(rest % a.n_mom_grp);
        const int g = (int)(rest / a.n_mom_grp);
        const int cb = g * blocks_per_group + c / kBlockCols;
        const int cc = c % kBlockCols;
        double sx = 0.0, sy = 0.0;
        for (int ch = 0; ch < a.n_chunks; ++ch) {
            const double2 v =
                a.partial[(((size_t)ch * a.n_colblocks + cb) * a.n_mom_grp + m) * kBlockCols + cc];
            sx += v.x;
            sy += v.y;
        }
        const size_t G = (size_t)(g / a.inner) * a.outer_stride + a.off + g % a.inner;
        a.out[(G * a.n_mom_total + a.m_off + m) * (size_t)a.group_cols + c] = make_double2(sx, sy);
    }
}

// ---------------------------------------------------------------------------
// Combine: C[pair][tau][op][s][t] = sum_i w_i sum_c S_i(p')[s][c] I_i(q,tau)[op][t][c]
// One workgroup per (pair, tau, op) x 64-row spectator block; 256 threads, each
// a 4x4 block of the 64x64 output tile.  FP64 throughout.
// ---------------------------------------------------------------------------
constexpr int kCombNoiseChunk = 4;

__global__ void __launch_bounds__(256) combine_kernel(CombineArgs a) {
    __shared__ double2 sA[kCombNoiseChunk * 3][64];
    __shared__ double2 sB[kCombNoiseChunk * 3][64];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int sb = blockIdx.y;
    size_t rest = blockIdx.x;
    const int o = (int)(rest % a.n_sel);
    rest /= a.n_sel;
    const int tau = (int)(rest % a.n_tau);
    const int pr = (int)(rest / a.n_tau);
    int p, q;
    if (a.pairs) {
        p = a.pairs[2 * pr];
        q = a.pairs[2 * pr + 1];
    } else {
        p = pr / a.n_q;
        q = pr % a.n_q;
    }
    const int op = a.op_begin + o;
    const size_t spin3 = (size_t)a.spin * 3;

    double2 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);

    for (int i0 = 0; i0 < a.n_noise; i0 += kCombNoiseChunk) {
        const int nc = min(kCombNoiseChunk, a.n_noise - i0);
        __syncthreads();
        for (int e = tid; e < nc * 3 * 64; e += 256) {
            const int kk = e >> 6, x = e & 63;
            const int i = i0 + kk / 3, c = kk % 3;
            const double w = a.w[i];
            const double2 sv = a.S[((size_t)i * a.n_p + p) * spin3 + (size_t)(sb * 64 + x) * 3 + c];
            sA[kk][x] = make_double2(w * sv.x, w * sv.y);
            sB[kk][x] = a.I[((((size_t)i * a.n_tau + tau) * a.n_ops + op) * a.n_q + q) * kBlockCols +
                            x * 3 + c];
        }
        __syncthreads();
        for (int kk = 0; kk < nc * 3; ++kk) {
            double2 av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = sA[kk][ty + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = sB[kk][tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[i][j].x = fma(av[i].x, bv[j].x, fma(-av[i].y, bv[j].y, acc[i][j].x));
                    acc[i][j].y = fma(av[i].x, bv[j].y, fma(av[i].y, bv[j].x, acc[i][j].y));
                }
        }
    }
    double2* out = a.out + ((((size_t)pr * a.n_tau + tau) * a.n_sel + o) * a.spin + (size_t)sb * 64) * 64;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) out[(size_t)(ty + 16 * i) * 64 + tx + 16 * j] = acc[i][j];
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
namespace {

template <typename R, int KT, int MTMAX, int WM, int WN, int CT, template <typename, int, int> class ProdT>
hipError_t launch_proj(const ProjGrid& pg, const typename ProdT<R, KT, 64 * WM * WN>::Args& a,
                       hipStream_t st) {
    dim3 grid(pg.n_colblocks, pg.n_chunks);
    dim3 block(64 * WM * WN);
    hipLaunchKernelGGL((proj_kernel<R, KT, MTMAX, WM, WN, CT, ProdT>), grid, block, 0, st, pg, a);
    return hipGetLastError();
}

template <template <typename, int, int> class ProdT>
hipError_t dispatch(bool f64, int mt, const ProjGrid& pg, const typename ProdT<float, 32, 256>::Args& a,
                    hipStream_t st) {
    if (f64) {
        if (mt <= 4) return launch_proj<double, 16, 4, 1, 4, 3, ProdT>(pg, a, st);
        return hipErrorInvalidValue;
    }
    if (mt <= 4) return launch_proj<float, 32, 4, 1, 4, 3, ProdT>(pg, a, st);
    if (mt <= 8) return launch_proj<float, 32, 8, 2, 4, 3, ProdT>(pg, a, st);
    if (mt <= 12) return launch_proj<float, 32, 12, 2, 4, 3, ProdT>(pg, a, st);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_spectator_meson(bool f64, int mt, const ProjGrid& pg, const MesonSpecArgs& a,
                                  hipStream_t st) {
    return dispatch<MesonSpecProducer>(f64, mt, pg, a, st);
}

hipError_t launch_spectator_baryon(bool f64, int mt, const ProjGrid& pg, const BaryonSpecArgs& a,
                                   hipStream_t st) {
    return dispatch<BaryonSpecProducer>(f64, mt, pg, a, st);
}

hipError_t launch_insertion(bool f64, int mt, const ProjGrid& pg, const InsertionArgs& a,
                            hipStream_t st) {
    return dispatch<InsertionProducer>(f64, mt, pg, a, st);
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st) {
    const size_t total = (size_t)a.n_groups * a.n_mom_grp * a.group_cols;
    size_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_combine(const CombineArgs& a, hipStream_t st) {
    dim3 grid((unsigned)((size_t)a.n_pairs * a.n_tau * a.n_sel), a.spin / 64);
    hipLaunchKernelGGL(combine_kernel, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace c3pt
