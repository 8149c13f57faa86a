// Factored projection with the left-derivative producer of the symmetrized
// insertion, and the FP64 assembly <->D_nu = 1/2 (->D_nu - <-D_nu) in place.
#include "c3pt_fac.h"
#include "c3pt_fac_left.h"
#include "c3pt_analysis.h"

namespace c3pt {

hipError_t launch_fac_insertion_left(bool f64, bool acc, const ProjGrid& pg, const InsertionLeftArgs& a,
                                     hipStream_t st) {
    return launch_fac<FacInsLeftProd, false>(f64, acc, pg, a, st);
}

// out[noise][tau][op][m][192] with n_ops = 9: op 5 + nu holds <-D_nu on entry
// and 1/2 (->D_nu - <-D_nu) on exit; ->D_nu is op 1 + nu.
__global__ void __launch_bounds__(256) symmetrize_kernel(double2* out, long long n_outer, int n_mom) {
    const long long per = (long long)4 * n_mom * 192;   // values of the four nu of one (noise, tau)
    const long long total = n_outer * per;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const long long o = i / per, w = i - o * per;
        double2* base = out + o * (long long)9 * n_mom * 192;
        const double2 r = base[(long long)n_mom * 192 + w];        // ops 1..4
        double2& l = base[(long long)5 * n_mom * 192 + w];         // ops 5..8
        l = make_double2(0.5 * (r.x - l.x), 0.5 * (r.y - l.y));
    }
}

hipError_t launch_symmetrize(double2* out, long long n_outer, int n_mom, hipStream_t st) {
    const long long total = n_outer * 4 * n_mom * 192;
    const unsigned blocks = (unsigned)std::min<long long>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(symmetrize_kernel, dim3(blocks), dim3(256), 0, st, out, n_outer, n_mom);
    return hipGetLastError();
}

// n_ops = 37: out[o][op][w] (37 operators) from the 53 internal ones in[o][op][w]:
// ops 0..20 copied; op 21 + 4 mu + nu = 1/4 (D_mu D_nu - mixed(mu, nu) - mixed(nu, mu) + left-left(mu, nu)),
// with D_mu D_nu = internal op 5 + 4 nu + mu, mixed(mu, nu) = 21 + 4 mu + nu, left-left = 37 + 4 mu + nu.
__global__ void __launch_bounds__(256) assemble_sym2_kernel(const double2* in, double2* out, long long n_outer,
                                                            int n_mom) {
    const long long per = (long long)n_mom * 192;
    const long long total = n_outer * 37 * per;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const long long w = i % per, r = i / per;
        const int op = (int)(r % 37);
        const long long o = r / 37;
        const double2* b = in + o * 53 * per + w;
        double2 v;
        if (op < 21) {
            v = b[op * per];
        } else {
            const int mu = (op - 21) / 4, nu = (op - 21) % 4;
            const double2 rr = b[(5 + 4 * nu + mu) * per], lr = b[(21 + 4 * mu + nu) * per];
            const double2 rl = b[(21 + 4 * nu + mu) * per], ll = b[(37 + 4 * mu + nu) * per];
            v = make_double2(0.25 * (rr.x - lr.x - rl.x + ll.x), 0.25 * (rr.y - lr.y - rl.y + ll.y));
        }
        out[i] = v;
    }
}

hipError_t launch_assemble_sym2(const double2* in, double2* out, long long n_outer, int n_mom, hipStream_t st) {
    const long long total = n_outer * 37 * n_mom * 192;
    const unsigned blocks = (unsigned)std::min<long long>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(assemble_sym2_kernel, dim3(blocks), dim3(256), 0, st, in, out, n_outer, n_mom);
    return hipGetLastError();
}

}  // namespace c3pt
