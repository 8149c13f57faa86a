// Phase tables of the momentum projection.
//
// phi_m(x) = exp(sigma * 2 pi i * sum_j k_mj (x_j - r_j) / L_j)   (Eqs. (9)-(10),
// with the source offset of Sec. 2.1).  The phase index is exact integer
// arithmetic: num = sum_j k_j (x_j - r_j) * (V3 / L_j) mod V3 and
// phi = exp(sigma * 2 pi i num / V3), evaluated with FP64 sincospi.
//
// A table is built once per (geometry, source, sign, momentum group, layout)
// and reused by every projection launch with that key; it is laid out exactly
// as the consumer stages it in LDS, so the fused kernel copies one contiguous
// block per site tile instead of evaluating phases.
#include "c3pt_device.h"

namespace c3pt {

namespace {

__device__ __forceinline__ void phase_value(const PhaseSpec& ph, int V3, int site, int m, double& re, double& im) {
    const int L1 = ph.L[0], L2 = ph.L[1], L3 = ph.L[2];
    const int x1 = site % L1, x2 = (site / L1) % L2, x3 = site / (L1 * L2);
    const long long d1 = (x1 - ph.r[0] + L1) % L1, d2 = (x2 - ph.r[1] + L2) % L2, d3 = (x3 - ph.r[2] + L3) % L3;
    const long long n = (long long)ph.k[0][m] * d1 * (long long)(L2 * L3) +
                        (long long)ph.k[1][m] * d2 * (long long)(L1 * L3) +
                        (long long)ph.k[2][m] * d3 * (long long)(L1 * L2);
    const long long num = n % (long long)V3;
    double s, c;
    sincospi(2.0 * (double)num / (double)V3, &s, &c);
    re = c;
    im = ph.sigma * s;
}

template <typename R>
__global__ void __launch_bounds__(256) phase_native_kernel(PhaseSpec ph, int V3, int Vpad, int mrows, C2<R>* out) {
    const size_t total = (size_t)Vpad * mrows;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int site = (int)(idx / mrows), m = (int)(idx % mrows);
        C2<R> v = {0, 0};
        if (site < V3 && m < ph.n_mom) {
            double re, im;
            phase_value(ph, V3, site, m, re, im);
            v = {(R)re, (R)im};
        }
        out[idx] = v;
    }
}

// A operand of the 16x16x32 MFMA for 16-site block b, row tile rt, lane
// 16*g + r, element e: row r = (momentum 8*rt + r/2, part r&1), site
// 16*b + 4*g + e/2, component e&1; real row (phi_re, -phi_im), imaginary
// row (phi_im, phi_re); each value split into hi + lo.
template <typename T16>
__global__ void __launch_bounds__(256) phase_split_kernel(PhaseSpec ph, int V3, int Vpad, int mtmax, T16* out) {
    const int mrows = 8 * mtmax;
    const size_t total = (size_t)Vpad * mrows;
    const size_t blk_elems = (size_t)2 * mtmax * 64 * 8;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int site = (int)(idx / mrows), m = (int)(idx % mrows);
        double re = 0.0, im = 0.0;
        if (site < V3 && m < ph.n_mom) phase_value(ph, V3, site, m, re, im);
        const int b = site >> 4, jj = site & 15, g = jj >> 2, e0 = 2 * (jj & 3);
        const int rt = m >> 3, r = 2 * (m & 7);
        T16* hi = out + (size_t)b * blk_elems + (size_t)rt * 64 * 8;
        T16* lo = hi + (size_t)mtmax * 64 * 8;
        auto put = [&](int lane, int e, float x) {
            const T16 h = (T16)x;
            hi[lane * 8 + e] = h;
            lo[lane * 8 + e] = (T16)(x - (float)h);
        };
        const float fr = (float)re, fi = (float)im;
        put(16 * g + r, e0, fr);          // real row, re component
        put(16 * g + r, e0 + 1, -fi);     // real row, im component
        put(16 * g + r + 1, e0, fi);      // imaginary row, re component
        put(16 * g + r + 1, e0 + 1, fr);  // imaginary row, im component
    }
}

int vpad(int V3) { return (V3 + 31) / 32 * 32; }

}  // namespace

// Bytes per (site, momentum row): one complex value (FP64: 16, FP32: 8), or in
// the split layout four A-operand values x (hi, lo) x 2 bytes = 16.
size_t phase_table_bytes(int mode, int V3, int mtmax) {
    const size_t rows = (size_t)vpad(V3) * 8 * mtmax;
    switch (mode) {
        case kModeF64: return rows * 16;
        case kModeF32: return rows * 8;
        default: return rows * 16;
    }
}

hipError_t launch_phase_table(int mode, const PhaseSpec& ph, int V3, int mtmax, void* out, hipStream_t st) {
    const int Vp = vpad(V3);
    const size_t total = (size_t)Vp * 8 * mtmax;
    const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 65536);
    switch (mode) {
        case kModeF64:
            hipLaunchKernelGGL(phase_native_kernel<double>, dim3(blocks), dim3(256), 0, st, ph, V3, Vp, 8 * mtmax,
                               (C2<double>*)out);
            break;
        case kModeF32:
            hipLaunchKernelGGL(phase_native_kernel<float>, dim3(blocks), dim3(256), 0, st, ph, V3, Vp, 8 * mtmax,
                               (C2<float>*)out);
            break;
        case kModeSplitBF16:
            hipLaunchKernelGGL(phase_split_kernel<__bf16>, dim3(blocks), dim3(256), 0, st, ph, V3, Vp, mtmax,
                               (__bf16*)out);
            break;
        case kModeSplitF16:
            hipLaunchKernelGGL(phase_split_kernel<_Float16>, dim3(blocks), dim3(256), 0, st, ph, V3, Vp, mtmax,
                               (_Float16*)out);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace c3pt
