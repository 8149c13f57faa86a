// Internal declarations shared by the host API and the kernels of libc3pt.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace c3pt {

// One column block of the projection GEMM = one 192-component spin-colour group.
constexpr int kBlockCols = 192;
// Largest momentum group handled by one projection launch (FP32 / FP64).
constexpr int kMaxMomGroupF32 = 96;
constexpr int kMaxMomGroupF64 = 32;
constexpr int kMaxMomGroup = 128;
// Largest number of insertion timeslices per launch (pointer tables travel as
// kernel arguments).
constexpr int kMaxTauPerLaunch = 24;
// FP32 partial sums never run over more sites than this before they are
// handed to the FP64 reduction.
constexpr int kMaxSitesPerChunkF32 = 2048;
constexpr int kMaxL = 256;

// Momentum list and phase convention of one projection launch.
struct PhaseSpec {
    int L[3];
    int r[3];          // source position, already reduced into [0, L_j)
    int sigma;         // -1 spectator, +1 insertion
    int cubic;         // L1 == L2 == L3: single-table phase lookup
    int n_mom;         // momenta in this group
    uint8_t k[3][kMaxMomGroup];   // components reduced into [0, L_j)
};

struct ProjGrid {
    PhaseSpec ph;
    int V3;
    int chunk_sites;   // sites per split-site chunk (multiple of the site tile)
    int n_chunks;
    int n_colblocks;
    double2* partial;  // [n_chunks][n_colblocks][n_mom][192] FP64 partial sums
};

// Producer arguments -------------------------------------------------------
struct MesonSpecArgs {
    const void* G;     // [144][V3]
    const void* eta;   // [N][12][V3]
};

struct BaryonSpecArgs {
    const void* G1;
    const void* G2;
    const void* eta;
};

struct InsertionArgs {
    int n_tau;         // timeslices in this launch
    int n_ops;         // 1 or 5
    int n_noise;
    const void* G[kMaxTauPerLaunch];     // G(tau)
    const void* Gn[kMaxTauPerLaunch];    // G(tau+1)  (derivative ops only)
    const void* Gp[kMaxTauPerLaunch];    // G(tau-1)
    const void* s[kMaxTauPerLaunch];     // s(tau) [N][12][V3]
    const void* U[kMaxTauPerLaunch];     // U(tau) [4][3][3][V3]
    const void* Up[kMaxTauPerLaunch];    // U(tau-1)
};

// Reduction of the split-site partial sums: output[G][m][c], c < group_cols,
// with output group G = (g / inner) * outer_stride + off + g % inner for the
// launch-local group g (this places a subset of insertion timeslices).
struct ReduceArgs {
    const double2* partial;
    double2* out;
    int n_chunks;
    int n_colblocks;
    int n_groups;      // launch-local groups
    int group_cols;    // 192 or 3072
    int n_mom_grp;     // momenta in this group
    int n_mom_total;   // momenta in the output
    int m_off;         // first momentum of this group in the output
    int inner, outer_stride, off;
};

struct CombineArgs {
    const double2* S;     // [N][n_p][spin*3]
    const double2* I;     // [N][n_tau][n_ops][n_q][192]
    const double* w;      // device [N]
    const int* pairs;     // device [n_pairs][2] or null (all pairs)
    double2* out;         // [n_pairs][n_tau][n_sel][spin][64]
    int n_noise, n_p, n_q, n_tau, n_ops, op_begin, n_sel, spin, n_pairs;
};

// Launchers (defined in c3pt_kernels.hip). They return hipError_t of the launch.
hipError_t launch_spectator_meson(bool f64, int mt, const ProjGrid& pg, const MesonSpecArgs& a,
                                  hipStream_t st);
hipError_t launch_spectator_baryon(bool f64, int mt, const ProjGrid& pg, const BaryonSpecArgs& a,
                                   hipStream_t st);
hipError_t launch_insertion(bool f64, int mt, const ProjGrid& pg, const InsertionArgs& a,
                            hipStream_t st);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st);
hipError_t launch_combine(const CombineArgs& a, hipStream_t st);

}  // namespace c3pt
