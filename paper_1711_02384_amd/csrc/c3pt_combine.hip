// FP64 kernels of libc3pt: the deterministic reduction of split-site partial
// sums (single calls and batches) and the noise-weighted combine of spectator
// and insertion parts.
#include "c3pt_device.h"

namespace c3pt {

// exp(-sigma 2 pi i k.r / L) for momentum k (components reduced mod L_j):
// the phase origin moved from 0 to the source position r.
__device__ __forceinline__ double2 source_factor(const int (&L)[3], const int (&r)[3], int sigma, int k1, int k2,
                                                 int k3) {
    const long long V3 = (long long)L[0] * L[1] * L[2];
    const long long n = (long long)k1 * r[0] * (L[1] * L[2]) + (long long)k2 * r[1] * (L[0] * L[2]) +
                        (long long)k3 * r[2] * (L[0] * L[1]);
    double s, c;
    sincospi(2.0 * (double)(n % V3) / (double)V3, &s, &c);
    return make_double2(c, -sigma * s);
}

__device__ __forceinline__ double2 cmul_d(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reduction of the split-site partial sums, times the
// source factor of each momentum.
// ---------------------------------------------------------------------------
// Each thread sums one output element over the chunks in a fixed order: eight
// interleaved FP64 partial sums (chunk ch into sum ch % 8, so eight loads are
// in flight), combined pairwise at the end.  Index arithmetic is 32-bit (the
// launcher takes the 64-bit form when an index would not fit).
template <typename P2, typename I>
__global__ void __launch_bounds__(256) reduce_kernel(ReduceArgs a) {
    const I total = (I)a.n_groups * (I)a.n_mom_grp * (I)a.group_cols;
    const int blocks_per_group = a.group_cols / kBlockCols;
    const P2* partial = (const P2*)a.partial;
    const size_t cstride = (size_t)a.n_colblocks * a.n_mom_grp * kBlockCols;   // elements between chunks
    for (I idx = (I)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (I)gridDim.x * blockDim.x) {
        const int c = (int)(idx % (I)a.group_cols);
        const I rest = idx / (I)a.group_cols;
        const int m = (int)(rest % (I)a.n_mom_grp);
        const int g = (int)(rest / (I)a.n_mom_grp);
        const int cb = g * blocks_per_group + c / kBlockCols;
        const int cc = c % kBlockCols;
        const P2* p = partial + ((size_t)cb * a.n_mom_grp + m) * kBlockCols + cc;
        double sx[8], sy[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) sx[k] = sy[k] = 0.0;
        int ch = 0;
        for (; ch + 8 <= a.n_chunks; ch += 8) {
            P2 v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = p[(size_t)(ch + k) * cstride];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                sx[k] += (double)v[k].x;
                sy[k] += (double)v[k].y;
            }
        }
#pragma unroll
        for (int k = 0; k < 7; ++k)
            if (ch + k < a.n_chunks) {
                const P2 v = p[(size_t)(ch + k) * cstride];
                sx[k] += (double)v.x;
                sy[k] += (double)v.y;
            }
        const double tx = ((sx[0] + sx[1]) + (sx[2] + sx[3])) + ((sx[4] + sx[5]) + (sx[6] + sx[7]));
        const double ty = ((sy[0] + sy[1]) + (sy[2] + sy[3])) + ((sy[4] + sy[5]) + (sy[6] + sy[7]));
        const double2 f = source_factor(a.ph.L, a.ph.r, a.ph.sigma, a.ph.k[0][m], a.ph.k[1][m], a.ph.k[2][m]);
        const size_t G = (size_t)(g / a.inner) * a.outer_stride + a.off + g % a.inner;
        a.out[(G * a.n_mom_total + a.m_off + m) * (size_t)a.group_cols + c] = cmul_d(f, make_double2(tx, ty));
    }
}

// ---------------------------------------------------------------------------
// Batched reduction: thread per output element of any job of the group.  The
// job of an element is found by binary search in the prefix sums.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) batch_reduce_kernel(BatchReduceArgs a, long long total) {
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        int lo = 0, hi = a.n_jobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.out_offset[mid] <= idx) lo = mid;
            else hi = mid - 1;
        }
        const BatchJob& job = a.jobs[lo];
        const long long e = idx - a.out_offset[lo];
        const int gc = job.group_cols;
        const int n_mom = job.n_mom;
        const int c = (int)(e % gc);
        const long long rest = e / gc;
        const int m = (int)(rest % n_mom);
        const int g = (int)(rest / n_mom);
        const int cb = g * (gc / kBlockCols) + c / kBlockCols;
        const int cc = c % kBlockCols;
        const float2* partial = (const float2*)job.partial;
        double sx = 0.0, sy = 0.0;
        for (int ch = 0; ch < job.n_chunks; ++ch) {
            const float2 v = partial[(((size_t)ch * job.n_colblocks + cb) * n_mom + m) * kBlockCols + cc];
            sx += (double)v.x;
            sy += (double)v.y;
        }
        int k[3];
        for (int j = 0; j < 3; ++j) {
            const int L = job.L[j];
            k[j] = ((job.k[3 * m + j] % L) + L) % L;
        }
        const double2 f = source_factor(job.L, job.r, job.sigma, k[0], k[1], k[2]);
        const long long G = (long long)(g / job.out_inner) * job.out_stride + job.out_off + g % job.out_inner;
        job.out[(G * n_mom + m) * gc + c] = cmul_d(f, make_double2(sx, sy));
    }
}

__global__ void reset_kernel(int* counters, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) counters[i] = 0;
}

// ---------------------------------------------------------------------------
// Combine: C[pair][tau][op][s][t] = sum_i w_i sum_c S_i(p')[s][c] I_i(q,tau)[op][t][c]
// One workgroup per (pair, tau, op) x 64-row spectator block: a 64 x 64
// complex GEMM over K = (noise, colour).  The weighted spectator rows and the
// insertion columns of four noise vectors at a time are staged in LDS; each
// of the four waves owns a 32 x 32 quadrant as 2 x 2 tiles of the FP64 MFMA
// 16x16x4, with the complex product as four real products
// (re += ar br - ai bi, im += ar bi + ai br).  FP64 throughout.
// ---------------------------------------------------------------------------
constexpr int kCombNoiseChunk = 4;
constexpr int kCombK = kCombNoiseChunk * 3;   // staged K entries (a multiple of the MFMA's 4)

__global__ void __launch_bounds__(256) combine_kernel(CombineArgs a) {
    using MF = Mfma<double>;
    using acc_t = MF::acc_t;
    __shared__ double2 sA[kCombK][64];
    __shared__ double2 sB[kCombK][64];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int r0 = (wave >> 1) * 32, c0 = (wave & 1) * 32;   // the wave's quadrant
    const int li = lane & 15, lk = lane >> 4;
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
    const int n_tau_in = a.n_tau_in > 0 ? a.n_tau_in : a.n_tau;

    acc_t cr[2][2], ci[2][2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
            cr[ti][tj] = acc_t{0.0, 0.0, 0.0, 0.0};
            ci[ti][tj] = acc_t{0.0, 0.0, 0.0, 0.0};
        }

    for (int i0 = 0; i0 < a.n_noise; i0 += kCombNoiseChunk) {
        const int nk = min(kCombNoiseChunk, a.n_noise - i0) * 3;
        __syncthreads();
        // K entries past the last noise vector are zero
        for (int e = tid; e < kCombK * 64; e += 256) {
            const int kk = e >> 6, x = e & 63;
            double2 av = make_double2(0.0, 0.0), bv = make_double2(0.0, 0.0);
            if (kk < nk) {
                const int i = i0 + kk / 3, c = kk % 3;
                const double w = a.w[i];
                const double2 sv = a.S[((size_t)i * a.n_p + p) * spin3 + (size_t)(sb * 64 + x) * 3 + c];
                av = make_double2(w * sv.x, w * sv.y);
                bv = a.I[((((size_t)i * n_tau_in + a.tau0 + tau) * a.n_ops + op) * a.n_q + q) * kBlockCols + x * 3 + c];
            }
            sA[kk][x] = av;
            sB[kk][x] = bv;
        }
        __syncthreads();
        for (int k0 = 0; k0 < nk; k0 += 4) {
            // A operand: row li of the tile, K entry k0 + lk; B: column li, K entry k0 + lk
            double2 av[2], bv[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                av[t] = sA[k0 + lk][r0 + 16 * t + li];
                bv[t] = sB[k0 + lk][c0 + 16 * t + li];
            }
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj) {
                    cr[ti][tj] = MF::mac(av[ti].x, bv[tj].x, cr[ti][tj]);
                    cr[ti][tj] = MF::mac(-av[ti].y, bv[tj].y, cr[ti][tj]);
                    ci[ti][tj] = MF::mac(av[ti].x, bv[tj].y, ci[ti][tj]);
                    ci[ti][tj] = MF::mac(av[ti].y, bv[tj].x, ci[ti][tj]);
                }
        }
    }
    // the output is written once and not read again by this step: streaming
    // (non-temporal) stores keep it from displacing the inputs in the caches.
    // FP64 accumulator layout: register j of lane l holds row 4 j + l / 16,
    // column l % 16 of its tile.
    typedef double d2v __attribute__((ext_vector_type(2)));
    d2v* out = (d2v*)(a.out + ((((size_t)pr * a.n_tau + tau) * a.n_sel + o) * a.spin + (size_t)sb * 64) * 64);
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = r0 + 16 * ti + 4 * j + lk, col = c0 + 16 * tj + li;
                const d2v v = {cr[ti][tj][j], ci[ti][tj][j]};
                __builtin_nontemporal_store(v, &out[(size_t)row * 64 + col]);
            }
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st) {
    const size_t total = (size_t)a.n_groups * a.n_mom_grp * a.group_cols;
    size_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) blocks = 1;
    const bool small = total + (size_t)65536 * 256 < ((size_t)1 << 32);
    if (a.f64 && small)
        hipLaunchKernelGGL((reduce_kernel<double2, unsigned>), dim3((unsigned)blocks), dim3(256), 0, st, a);
    else if (a.f64)
        hipLaunchKernelGGL((reduce_kernel<double2, size_t>), dim3((unsigned)blocks), dim3(256), 0, st, a);
    else if (small)
        hipLaunchKernelGGL((reduce_kernel<float2, unsigned>), dim3((unsigned)blocks), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((reduce_kernel<float2, size_t>), dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_batch_reduce(const BatchReduceArgs& a, long long total, hipStream_t st) {
    long long blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(batch_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a, total);
    return hipGetLastError();
}

hipError_t launch_reset(int* counters, int n, hipStream_t st) {
    hipLaunchKernelGGL(reset_kernel, dim3((n + 255) / 256), dim3(256), 0, st, counters, n);
    return hipGetLastError();
}

hipError_t launch_combine(const CombineArgs& a, hipStream_t st) {
    dim3 grid((unsigned)((size_t)a.n_pairs * a.n_tau * a.n_sel), a.spin / 64);
    hipLaunchKernelGGL(combine_kernel, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace c3pt
