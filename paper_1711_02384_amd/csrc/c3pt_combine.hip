// FP64 kernels of libc3pt: the deterministic reduction of split-site partial
// sums and the noise-weighted combine of spectator and insertion parts.
#include "c3pt_device.h"

namespace c3pt {

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
