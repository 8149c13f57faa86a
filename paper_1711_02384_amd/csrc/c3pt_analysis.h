// Analysis stage of the spin-open data: Gamma channels of the combine output.
#ifndef C3PT_ANALYSIS_H
#define C3PT_ANALYSIS_H

#include <vector>

#include "c3pt_internal.h"

namespace c3pt {

// Analysis stage (Gamma channels of the combine output).
constexpr int kMaxNucProj = 16;
struct GammaMesonArgs {
    const double2* C;      // [n_blk][64][64]: rows (b', a', a), columns (at, bt, b)
    const double2* mats;   // device [3][16][16]: Gsnk, Gins, Gsrc as [n][4x4 row-major]
    double2* out;          // [n_blk][n_snk][n_ins][n_src]
    int n_blk, n_snk, n_ins, n_src;
};
struct GammaNucleonArgs {
    const double2* C;      // [n_blk][1024][64]: rows (a1', a1, a2', a2, b'), columns (at, bt, b)
    const int* rows;       // device [n_rows]: rows with a non-zero weight
    const double2* w;      // device [n_rows][n_proj][4]: weight of (row, projector, b)
    const double2* gins;   // device [n_ins][16]
    double2* out;          // [n_blk][n_proj][n_ins]
    int n_blk, n_rows, n_proj, n_ins;
};
hipError_t launch_gamma_meson(const GammaMesonArgs& a, hipStream_t st);
hipError_t launch_gamma_nucleon(const GammaNucleonArgs& a, hipStream_t st);
// which = 0, 1: Gamma_n = g1^b0 g2^b1 g3^b2 g4^b3 (n = b0 + 2 b1 + 4 b2 + 8 b3);
// 2: gamma4 Gamma_n^dag gamma4.  out: [16][16] complex, row-major 4x4 each.
void gamma_default_matrices(int which, double2* out);
// Rows and weights of the nucleon channel (0: d current, 1: u current) for the
// diquark matrices A, Abar and projectors P (host [4x4] complex, NULL: C gamma5,
// gamma4 A^dag gamma4, (1 +- gamma4)/2).
void nucleon_weights(int channel, const double* A, const double* Abar, const double* P, int n_proj,
                     std::vector<int>* rows, std::vector<double2>* w);

// Symmetrized derivative insertion (n_ops = 9): the left-derivative launch and
// the in-place assembly of ops 5..8 from ops 1..4 (out: [n_outer][9][n_mom][192]).
struct InsertionLeftArgs;
hipError_t launch_fac_insertion_left(bool f64, bool acc, const ProjGrid& pg, const InsertionLeftArgs& a,
                                     hipStream_t st);
hipError_t launch_symmetrize(double2* out, long long n_outer, int n_mom, hipStream_t st);
// n_ops = 37: the 37 operators [n_outer][37][n_mom][192] from the 53 internal ones.
hipError_t launch_assemble_sym2(const double2* in, double2* out, long long n_outer, int n_mom, hipStream_t st);

// Gauge-covariant smearing step of colour vectors [n_outer][3][n_inner][V3].
struct SmearArgs {
    const void* in;
    void* out;
    const void* U;          // [4][3][3][V3] links of the timeslice (j = 0..2 used)
    int L[3], V3;
    int n_outer, n_inner;
    double norm;            // 1 / (1 + 6 kappa)
    double kappa_norm;      // kappa / (1 + 6 kappa)
    int vb_per_item;        // 8-vector blocks one workgroup runs on its tile (set by launch_smear)
};
hipError_t launch_smear(bool f64, const SmearArgs& a, hipStream_t st);

// One covariant derivative of a colour-vector field (two-derivative
// insertion operators): out = 1/2 [U_rho(x) fp(x+rho) - U_rho(x-rho)^dag fm(x-rho)].
struct DerivStencilArgs {
    const void* fp;         // field read at x + rho (time: the slice above)
    const void* fm;         // field read at x - rho (time: the slice below)
    const void* U;          // links [4][3][3][V3] giving U_rho(x)
    const void* Um;         // links giving U_rho(x - rho) (time: the slice below; spatial: = U)
    void* out;
    int L[3], V3;
    int n_outer, n_inner;
    int rho;
};
hipError_t launch_cov_deriv(bool f64, const DerivStencilArgs& a, hipStream_t st);

}  // namespace c3pt

#endif
