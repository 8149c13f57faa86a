// Analysis stage of the spin-open data: the combine output contracted with
// source, sink and insertion spin matrices.  The spins stay open through the
// measurement (Eqs. (9)-(10)) precisely so that every Gamma structure of
// Eq. (1) at source, sink and insertion follows afterwards (Sec. 1, Sec. 3).
//
// Meson: out[i][j][l] = sum Gsnk_i[a'][b'] Gins_j[at][bt] Gsrc_l[b][a] C[b'][a'][a][at][bt][b]
// as three 4x4 contractions, intermediates in LDS and the matrices read
// with workgroup-uniform addresses (scalar loads).  Nucleon: the proton's Wick terms (the
// diquark matrix at sink and source, a projector between the nucleon spins)
// become one weight per (row, b) of the [1024][64] data, built on the host;
// the kernel streams the weighted rows and applies Gins last.
#include "c3pt_analysis.h"
#include "c3pt_device.h"

#include <algorithm>
#include <array>
#include <complex>
#include <vector>

namespace c3pt {

namespace {

__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {
    c.x = fma(a.x, b.x, c.x);
    c.x = fma(-a.y, b.y, c.x);
    c.y = fma(a.x, b.y, c.y);
    c.y = fma(a.y, b.x, c.y);
    return c;
}

// Padded LDS strides (16-byte units): X1 rows [a][at bt b] with a stride of 68
// and 272 per sink matrix; X2 and the output stage with a stride of 17.
constexpr int kX1A = 68;
constexpr int kX1G = 4 * kX1A;
constexpr int kX2S = 17;

struct GammaMesonSmem {
    double2 X1[16 * kX1G];          // [g1][a][at bt b]; reused for the output stage
    double2 X2[256 * kX2S];         // [g1 g2][a b]
};

}  // namespace

__global__ void __launch_bounds__(256) gamma_meson_kernel(GammaMesonArgs a) {
    __shared__ GammaMesonSmem sm;
    const int tid = threadIdx.x;
    const double2* Cb = a.C + (size_t)blockIdx.x * 4096;
    // the matrices are read with workgroup-uniform addresses: scalar loads
    const double2* __restrict__ M = a.mats;
    // stage 1 (sink): thread = (a, at, bt, b); X1[g1] = sum_{a', b'} Gsnk[g1][a'][b'] C[b'][a'][.]
    double2 c[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) c[k] = Cb[k * 256 + tid];
    __syncthreads();
    const int x1off = (tid >> 6) * kX1A + (tid & 63);
    for (int g1 = 0; g1 < a.n_snk; ++g1) {
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int bp = 0; bp < 4; ++bp)
#pragma unroll
            for (int ap = 0; ap < 4; ++ap) s = cfma(M[g1 * 16 + ap * 4 + bp], c[bp * 4 + ap], s);
        sm.X1[g1 * kX1G + x1off] = s;
    }
    __syncthreads();
    // stage 2 (insertion): X2[g1 g2][a b] = sum_{at, bt} Gins[g2][at][bt] X1[g1][a][at][bt][b]
    for (int idx = tid; idx < a.n_snk * 16; idx += 256) {
        const int g1 = idx >> 4, ab = idx & 15, aa = ab >> 2, b = ab & 3;
        double2 x[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) x[k] = sm.X1[g1 * kX1G + aa * kX1A + k * 4 + b];
        for (int g2 = 0; g2 < a.n_ins; ++g2) {
            double2 s = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < 16; ++k) s = cfma(M[256 + g2 * 16 + k], x[k], s);
            sm.X2[(g1 * 16 + g2) * kX2S + ab] = s;
        }
    }
    __syncthreads();
    // stage 3 (source): out[g1][g2][g3] = sum_{a, b} Gsrc[g3][b][a] X2[g1 g2][a b]
    const int n12 = a.n_snk * a.n_ins;
    for (int idx = tid; idx < n12; idx += 256) {
        const int g1 = idx / a.n_ins, g2 = idx - g1 * a.n_ins;
        double2 y[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) y[k] = sm.X2[(g1 * 16 + g2) * kX2S + k];
        for (int g3 = 0; g3 < a.n_src; ++g3) {
            double2 s = make_double2(0.0, 0.0);
#pragma unroll
            for (int aa = 0; aa < 4; ++aa)
#pragma unroll
                for (int b = 0; b < 4; ++b) s = cfma(M[512 + g3 * 16 + b * 4 + aa], y[aa * 4 + b], s);
            sm.X1[idx * kX2S + g3] = s;
        }
    }
    __syncthreads();
    const int total = n12 * a.n_src;
    double2* ob = a.out + (size_t)blockIdx.x * total;
    for (int i = tid; i < total; i += 256) {
        const int r = i / a.n_src;
        ob[i] = sm.X1[r * kX2S + (i - r * a.n_src)];
    }
}

// One workgroup per block of nucleon data; wave w of kNucWaves takes rows w,
// w + kNucWaves, ..., four at a time (four row loads in flight); lane
// = (at, bt, b) reads one complex of the row (a row is 64 consecutive values).
// NP: the largest projector count of the instantiation (4 keeps the
// accumulators of the usual parity projectors in few registers).
constexpr int kNucWaves = 8;

template <int NP>
__global__ void __launch_bounds__(64 * kNucWaves) gamma_nucleon_kernel(GammaNucleonArgs a) {
    constexpr int NT = 64 * kNucWaves;
    __shared__ double2 Z[kNucWaves][NP][kX2S];
    __shared__ double2 Gi[16][16];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, b = lane & 3;
    for (int i = tid; i < a.n_ins * 16; i += NT) (&Gi[0][0])[i] = a.gins[i];
    const double2* Cb = a.C + (size_t)blockIdx.x * 65536 + lane;
    double2 acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = make_double2(0.0, 0.0);
    auto add_row = [&](int k, double2 v) {
        const double2* wk = a.w + (size_t)k * a.n_proj * 4 + b;
#pragma unroll
        for (int p = 0; p < NP; ++p)
            if (p < a.n_proj) acc[p] = cfma(wk[p * 4], v, acc[p]);
    };
    int k = wave;
    for (; k + 3 * kNucWaves < a.n_rows; k += 4 * kNucWaves) {
        double2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = Cb[(size_t)a.rows[k + u * kNucWaves] * 64];
#pragma unroll
        for (int u = 0; u < 4; ++u) add_row(k + u * kNucWaves, v[u]);
    }
    for (; k < a.n_rows; k += kNucWaves) add_row(k, Cb[(size_t)a.rows[k] * 64]);
    // sum the four lanes of one (at, bt): b is the lowest two bits of the lane
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        if (p < a.n_proj) {
            acc[p].x += __shfl_xor(acc[p].x, 1);
            acc[p].y += __shfl_xor(acc[p].y, 1);
            acc[p].x += __shfl_xor(acc[p].x, 2);
            acc[p].y += __shfl_xor(acc[p].y, 2);
            if (b == 0) Z[wave][p][lane >> 2] = acc[p];
        }
    }
    __syncthreads();
    const int total = a.n_proj * a.n_ins;
    double2* ob = a.out + (size_t)blockIdx.x * total;
    for (int i = tid; i < total; i += NT) {
        const int p = i / a.n_ins, j = i - p * a.n_ins;
        double2 s = make_double2(0.0, 0.0);
        for (int t = 0; t < 16; ++t) {
            double2 z = make_double2(0.0, 0.0);
#pragma unroll
            for (int w = 0; w < kNucWaves; ++w) {
                z.x += Z[w][p][t].x;
                z.y += Z[w][p][t].y;
            }
            s = cfma(Gi[j][t], z, s);
        }
        ob[i] = s;
    }
}

hipError_t launch_gamma_meson(const GammaMesonArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(gamma_meson_kernel, dim3((unsigned)a.n_blk), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gamma_nucleon(const GammaNucleonArgs& a, hipStream_t st) {
    if (a.n_proj <= 4)
        hipLaunchKernelGGL(gamma_nucleon_kernel<4>, dim3((unsigned)a.n_blk), dim3(64 * kNucWaves), 0, st, a);
    else
        hipLaunchKernelGGL(gamma_nucleon_kernel<kMaxNucProj>, dim3((unsigned)a.n_blk), dim3(64 * kNucWaves), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Host tables: DeGrand-Rossi gamma matrices and the proton's Wick terms.
// ---------------------------------------------------------------------------
namespace {

using M4 = std::array<std::complex<double>, 16>;

M4 mul(const M4& x, const M4& y) {
    M4 r{};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 4; ++k) r[i * 4 + j] += x[i * 4 + k] * y[k * 4 + j];
    return r;
}

M4 dagger(const M4& x) {
    M4 r{};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) r[i * 4 + j] = std::conj(x[j * 4 + i]);
    return r;
}

M4 identity() {
    M4 r{};
    for (int i = 0; i < 4; ++i) r[i * 5] = 1.0;
    return r;
}

// gamma_mu as (row, column, value) of its one non-zero per row
M4 gamma(int mu) {
    const std::complex<double> I(0.0, 1.0);
    M4 g{};
    switch (mu) {
        case 0: g[3] = I; g[6] = I; g[9] = -I; g[12] = -I; break;
        case 1: g[3] = -1.0; g[6] = 1.0; g[9] = 1.0; g[12] = -1.0; break;
        case 2: g[2] = I; g[7] = -I; g[8] = -I; g[13] = I; break;
        default: g[2] = 1.0; g[7] = 1.0; g[8] = 1.0; g[13] = 1.0; break;
    }
    return g;
}

M4 basis(int n) {
    M4 m = identity();
    for (int mu = 0; mu < 4; ++mu)
        if ((n >> mu) & 1) m = mul(m, gamma(mu));
    return m;
}

M4 creation(const M4& g) { return mul(mul(gamma(3), dagger(g)), gamma(3)); }

// Positions of the six non-insertion spins: the row (a1', a1, a2', a2, b')
// of the nucleon data and the source spin b of its column.
enum { kA1p = 0, kA1 = 1, kA2p = 2, kA2 = 3, kBp = 4, kB = 5 };
struct NucTerm {
    int sign;
    int snk[3];   // spins of (u_a, d_b, u_c) at the sink: A's two, then the nucleon spin
    int src[3];   // spins of (dbar_b, ubar_a, ubar_c) at the source: Abar's two, then the nucleon spin
};
// d current: spectators (G1, G2) = (u, u); the two u pairings.
const NucTerm kProtonD[] = {{+1, {kA1p, kBp, kA2p}, {kB, kA1, kA2}}, {+1, {kA1p, kBp, kA2p}, {kB, kA2, kA1}}};
// u current: spectators (G1, G2) = (u, d); the current on either u, from and to either u slot.
const NucTerm kProtonU[] = {{+1, {kBp, kA2p, kA1p}, {kA2, kB, kA1}}, {+1, {kBp, kA2p, kA1p}, {kA2, kA1, kB}},
                            {+1, {kA1p, kA2p, kBp}, {kA2, kB, kA1}}, {+1, {kA1p, kA2p, kBp}, {kA2, kA1, kB}}};

void put(const M4& m, double2* out) {
    for (int i = 0; i < 16; ++i) out[i] = make_double2(m[i].real(), m[i].imag());
}

M4 take(const double* p) {
    M4 m{};
    for (int i = 0; i < 16; ++i) m[i] = std::complex<double>(p[2 * i], p[2 * i + 1]);
    return m;
}

}  // namespace

void gamma_default_matrices(int which, double2* out) {
    for (int n = 0; n < 16; ++n) put(which == 2 ? creation(basis(n)) : basis(n), out + 16 * n);
}

void nucleon_weights(int channel, const double* A, const double* Abar, const double* P, int n_proj,
                     std::vector<int>* rows, std::vector<double2>* w) {
    const M4 Cg5 = mul(mul(gamma(1), gamma(3)), mul(mul(gamma(0), gamma(1)), mul(gamma(2), gamma(3))));
    const M4 mA = A ? take(A) : Cg5;
    const M4 mAb = Abar ? take(Abar) : creation(mA);
    std::vector<M4> mP;
    if (P) {
        for (int p = 0; p < n_proj; ++p) mP.push_back(take(P + 32 * p));
    } else {
        M4 plus = identity(), minus = identity();
        const M4 g4 = gamma(3);
        for (int i = 0; i < 16; ++i) {
            plus[i] = (plus[i] + g4[i]) * 0.5;
            minus[i] = (minus[i] - g4[i]) * 0.5;
        }
        mP = {plus, minus};
    }
    const NucTerm* terms = channel == 0 ? kProtonD : kProtonU;
    const int n_terms = channel == 0 ? 2 : 4;
    rows->clear();
    w->clear();
    std::vector<std::complex<double>> rw((size_t)n_proj * 4);
    for (int row = 0; row < 1024; ++row) {
        std::fill(rw.begin(), rw.end(), 0.0);
        bool any = false;
        for (int b = 0; b < 4; ++b) {
            const int v[6] = {(row >> 8) & 3, (row >> 6) & 3, (row >> 4) & 3, (row >> 2) & 3, row & 3, b};
            for (int t = 0; t < n_terms; ++t) {
                const NucTerm& T = terms[t];
                const std::complex<double> f = (double)T.sign * mA[v[T.snk[0]] * 4 + v[T.snk[1]]] *
                                               mAb[v[T.src[0]] * 4 + v[T.src[1]]];
                if (f == 0.0) continue;
                for (int p = 0; p < n_proj; ++p) {
                    const std::complex<double> x = f * mP[p][v[T.src[2]] * 4 + v[T.snk[2]]];
                    if (x != 0.0) {
                        rw[(size_t)p * 4 + b] += x;
                        any = true;
                    }
                }
            }
        }
        if (!any) continue;
        rows->push_back(row);
        for (auto& x : rw) w->push_back(make_double2(x.real(), x.imag()));
    }
}

}  // namespace c3pt
