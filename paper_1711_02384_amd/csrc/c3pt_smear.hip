// Gauge-covariant quark smearing of colour-vector fields on one timeslice
// (the paper smears the spectator's propagators at source and sink, Sec. 3;
// the operators of Sec. 2.1 may contain quark smearing).  One launch per step:
//   psi'(x) = [psi(x) + kappa sum_{j=1..3} (U_j(x) psi(x+j) + U_j(x-j)^dag psi(x-j))] / (1 + 6 kappa)
// Field layout [n_outer][3][n_inner][V3] (site fastest): the rows of a
// propagator slice (n_outer = 4 spins, n_inner = 12 columns) or noise and
// solution vectors (n_outer = 4 N, n_inner = 1).
//
// A workgroup takes 64 consecutive sites and a run of 8-vector blocks, one
// (site, vector) per thread and block: the six links of each site go to LDS
// once and serve every block of the run (the link bytes are read once per
// run, not once per 8 vectors); lanes run over sites, so every field read
// (centre and the six neighbours) is a coalesced row.  Work items are (site
// tile, run) with the tile fastest, dealt to the eight XCDs in contiguous
// ranges, so that the x2 / x3 neighbour rows a workgroup reads were mostly
// fetched into the same L2 by the tiles just before it.
#include "c3pt_device.h"
#include "c3pt_analysis.h"

namespace c3pt {

namespace {
constexpr int kSmSites = 64;
constexpr int kSmVecs = 8;
constexpr int kSmThreads = kSmSites * kSmVecs;   // one (site, vector) per thread
}  // namespace

template <typename R>
__global__ void __launch_bounds__(kSmThreads) smear_kernel(SmearArgs a) {
    __shared__ C2<R> uf[3][9][kSmSites];   // U_j(x)[c][d]
    __shared__ C2<R> ub[3][9][kSmSites];   // U_j(x - j)[c][d]
    const int tid = threadIdx.x;
    const int gx = (a.V3 + kSmSites - 1) / kSmSites;
    const int nw = gridDim.x, w = blockIdx.x;
    const int full = (nw / 8) * 8;
    const int item = (w < full) ? (w % 8) * (nw / 8) + w / 8 : w;
    const int tile = item % gx, run = item / gx;
    const int s0 = tile * kSmSites;
    const C2<R>* U = (const C2<R>*)a.U;
    const unsigned V3 = (unsigned)a.V3;
    const int L1 = a.L[0], L2 = a.L[1], L3 = a.L[2];
    // coordinates once per site; neighbours by compare and select (no
    // division per neighbour)
    struct Nbr {
        int p[3], m[3];
    };
    auto neighbours = [&](int n) {
        const int q = n / L1, x1 = n - q * L1, x3 = q / L2, x2 = q - x3 * L2;
        const int s2 = L1, s3 = L1 * L2;
        Nbr r;
        r.p[0] = n + (x1 == L1 - 1 ? 1 - L1 : 1);
        r.m[0] = n - (x1 == 0 ? 1 - L1 : 1);
        r.p[1] = n + (x2 == L2 - 1 ? (1 - L2) * s2 : s2);
        r.m[1] = n - (x2 == 0 ? (1 - L2) * s2 : s2);
        r.p[2] = n + (x3 == L3 - 1 ? (1 - L3) * s3 : s3);
        r.m[2] = n - (x3 == 0 ? (1 - L3) * s3 : s3);
        return r;
    };
    // links of the tile: thread (site i, direction j) among the first 192
    if (tid < 3 * kSmSites) {
        const int i = tid % kSmSites, j = tid / kSmSites;
        const int n = min(s0 + i, a.V3 - 1);
        const Nbr nb = neighbours(n);
        const int nmj = j == 0 ? nb.m[0] : (j == 1 ? nb.m[1] : nb.m[2]);
#pragma unroll
        for (int cd = 0; cd < 9; ++cd) {
            uf[j][cd][i] = U[(unsigned)(j * 9 + cd) * V3 + (unsigned)n];
            ub[j][cd][i] = U[(unsigned)(j * 9 + cd) * V3 + (unsigned)nmj];
        }
    }
    __syncthreads();
    const int i = tid % kSmSites;
    const int s = s0 + i;
    if (s >= a.V3) return;
    const Nbr nb = neighbours(s);
    int np[3], nm[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        np[j] = nb.p[j];
        nm[j] = nb.m[j];
    }
    const R norm = (R)a.norm, kn = (R)a.kappa_norm;
    const C2<R>* in = (const C2<R>*)a.in;
    C2<R>* out = (C2<R>*)a.out;
    const int n_vec = a.n_outer * a.n_inner;
    const int vb0 = run * a.vb_per_item;
    for (int vb = vb0; vb < vb0 + a.vb_per_item; ++vb) {
        const int v = vb * kSmVecs + tid / kSmSites;
        if (v >= n_vec) break;
        const int o = v / a.n_inner, in_i = v - o * a.n_inner;
        unsigned base[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) base[c] = (unsigned)((o * 3 + c) * a.n_inner + in_i) * V3;
        C2<R> hop[3] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C2<R> f[3], b[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                f[d] = in[base[d] + (unsigned)np[j]];
                b[d] = in[base[d] + (unsigned)nm[j]];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    hop[c] = cfma(hop[c], uf[j][c * 3 + d][i], f[d]);
                    hop[c] = cadd(hop[c], cmulc(b[d], ub[j][d * 3 + c][i]));   // conj(U(x-j)[d][c]) psi_d
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const C2<R> x = in[base[c] + (unsigned)s];
            out[base[c] + (unsigned)s] = C2<R>{norm * x.x + kn * hop[c].x, norm * x.y + kn * hop[c].y};
        }
    }
}

hipError_t launch_smear(bool f64, const SmearArgs& a0, hipStream_t st) {
    const long long gx = (a0.V3 + kSmSites - 1) / kSmSites;
    const long long gy = (a0.n_outer * (long long)a0.n_inner + kSmVecs - 1) / kSmVecs;
    // runs of vector blocks: about 2048 workgroups in all (at least one block each)
    const long long runs = std::max<long long>(1, std::min<long long>(gy, (2048 + gx - 1) / gx));
    SmearArgs a = a0;
    a.vb_per_item = (int)((gy + runs - 1) / runs);
    const long long n_runs = (gy + a.vb_per_item - 1) / a.vb_per_item;
    const dim3 grid((unsigned)(gx * n_runs));
    if (f64)
        hipLaunchKernelGGL(smear_kernel<double>, grid, dim3(kSmThreads), 0, st, a);
    else
        hipLaunchKernelGGL(smear_kernel<float>, grid, dim3(kSmThreads), 0, st, a);
    return hipGetLastError();
}

// One covariant derivative of a field of colour vectors (layout as above):
//   out(x) = 1/2 [U_rho(x) f(x + rho) - U_rho(x - rho)^dag f(x - rho)].
// Spatial rho: fp = fm = the slice, U = Um = U_rho of the slice, neighbours
// in the slice; time: fp, fm the adjacent slices at the same site, U = U_t of
// the slice, Um = U_t of the slice below.  One (site, vector) per thread; the
// two links of a site are read by the 8 vector threads of that site (cache).
template <typename R>
__global__ void __launch_bounds__(kSmThreads) cov_deriv_kernel(DerivStencilArgs a) {
    const int tid = threadIdx.x;
    const int gx = (a.V3 + kSmSites - 1) / kSmSites;
    const int nw = gridDim.x, w = blockIdx.x;
    const int full = (nw / 8) * 8;
    const int item = (w < full) ? (w % 8) * (nw / 8) + w / 8 : w;
    const int tile = item % gx, vb = item / gx;
    const int n = tile * kSmSites + tid % kSmSites;
    const int v = vb * kSmVecs + tid / kSmSites;
    if (n >= a.V3 || v >= a.n_outer * a.n_inner) return;
    const int L1 = a.L[0], L2 = a.L[1], L3 = a.L[2];
    int np = n, nm = n;
    if (a.rho < 3) {
        const int q = n / L1, x1 = n - q * L1, x3 = q / L2, x2 = q - x3 * L2;
        const int x = a.rho == 0 ? x1 : (a.rho == 1 ? x2 : x3);
        const int ext = a.rho == 0 ? L1 : (a.rho == 1 ? L2 : L3);
        const int st = a.rho == 0 ? 1 : (a.rho == 1 ? L1 : L1 * L2);
        np = n + (x == ext - 1 ? (1 - ext) * st : st);
        nm = n - (x == 0 ? (1 - ext) * st : st);
    }
    const unsigned V3 = (unsigned)a.V3;
    const int d = a.rho < 3 ? a.rho : 3;
    const C2<R>* U = (const C2<R>*)a.U + (size_t)d * 9 * V3;
    const C2<R>* Um = (const C2<R>*)a.Um + (size_t)d * 9 * V3;
    const C2<R>* fp = (const C2<R>*)a.fp;
    const C2<R>* fm = (const C2<R>*)a.fm;
    C2<R>* out = (C2<R>*)a.out;
    const int o = v / a.n_inner, in_i = v - o * a.n_inner;
    unsigned base[3];
    C2<R> f[3], b[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        base[c] = (unsigned)((o * 3 + c) * a.n_inner + in_i) * V3;
        f[c] = fp[base[c] + (unsigned)np];
        b[c] = fm[base[c] + (unsigned)nm];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        C2<R> acc = {0, 0};
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            acc = cfma(acc, U[(unsigned)(c * 3 + e) * V3 + (unsigned)n], f[e]);
            acc = csub(acc, cmulc(b[e], Um[(unsigned)(e * 3 + c) * V3 + (unsigned)nm]));
        }
        out[base[c] + (unsigned)n] = cscale(acc, (R)0.5);
    }
}

hipError_t launch_cov_deriv(bool f64, const DerivStencilArgs& a, hipStream_t st) {
    const long long gx = (a.V3 + kSmSites - 1) / kSmSites;
    const long long gy = (a.n_outer * (long long)a.n_inner + kSmVecs - 1) / kSmVecs;
    const dim3 grid((unsigned)(gx * gy));
    if (f64)
        hipLaunchKernelGGL(cov_deriv_kernel<double>, grid, dim3(kSmThreads), 0, st, a);
    else
        hipLaunchKernelGGL(cov_deriv_kernel<float>, grid, dim3(kSmThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace c3pt
