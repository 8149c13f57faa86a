// Host-side interface of the split-precision fused projection (c3pt_fs.hip).
#pragma once

#include "c3pt_internal.h"

namespace c3pt {

constexpr int kFsPlanes = 144;   // 3 summed colours x 48 B columns
constexpr int kFsPairsCB3 = 5;   // (k1, k2) pairs per k1 slot with three column blocks per workgroup

// Kernel arguments besides the grid.
//   kind 0: spectator (u = g eta), 1: insertion, local operator only,
//   kind 2: insertion with the nine slots (local, then (nu, +), (nu, -) for nu = x, y, z, t).
// B comes either from split blocks written by a pass before the launch (the
// nucleon diquark) or from FP32 propagator slices split in the kernel.
struct FsArgs {
    int L[3];
    int Lp, rows;          // padded row length of a split B block (multiple of KT), L2 * L3
    int N;                 // noise vectors of this launch: i_base .. i_base + N - 1 of the call
    int i_base;
    int n_share, n_slots;  // shares (timeslices of the launch; 1 for spectators), slots per share
    int colmap;            // 0: column at*48 + X; 1: nucleon (X/3)*12 + at*3 + X%3
    const void* B;         // split B source: blocks b_stride bytes apart; spectators: block = slot,
    size_t b_stride;       // insertion: block bidx[tau_j][role]
    int bidx[kMaxTauPerLaunch][3];
    const void* G[kMaxTauPerLaunch][3];   // FP32 B source: G(tau_j), G(tau_j + 1), G(tau_j - 1);
                                          // the meson spectator's (KIND 0) is conjugated with g[a'] g[a]
    const void* u0[kMaxTauPerLaunch];   // spectators: eta [N][12][V3] (entry 0); insertion: s(tau_j)
    const void* U[kMaxTauPerLaunch];    // U(tau_j) [4][3][3][V3]
    const void* Up[kMaxTauPerLaunch];   // U(tau_j - 1)
};

// Propagator slices -> split B blocks (fs_split_kernel), for launches that
// read each slice from many work items.
struct FsSplitArgs {
    int L[3];
    int Lp, rows;
    int n_slices;
    int conj_sign;         // meson spectator: conj(G) g[a'] g[a]
    const float2* G[kMaxTauPerLaunch + 2];
    void* out;             // [n_slices][rows][144][Lp/4] groups of four sites
};

// Nucleon diquark of (G1, G2) -> 16 split B blocks (fs_diquark_kernel).
struct FsDiquarkArgs {
    int L[3];
    int Lp, rows;
    const float2* G1;
    const float2* G2;
    void* out;             // [16][rows][144][Lp/4]
};

// FP64 reduction of an insertion launch with the nine derivative slots.
struct FsReduceArgs {
    const float2* partial;   // [n_chunks][n_colblocks][n_mom_grp][192], cb = (i * nt + j) * 9 + slot
    double2* out;            // [N][n_tau_total][5][n_mom_total][192]
    PhaseSpec ph;
    int n_chunks, n_colblocks;
    int N, nt, j0, n_tau_total;
    int n_mom_grp, n_mom_total, m_off;
};

// Site tile of the fused kernel for extents L: 32 when rows split into
// 32-site segments, else 16; rows are padded to a multiple of it.
inline int fs_kt(const int L[3]) { return L[0] % 32 == 0 ? 32 : 16; }
inline int fs_lp(const int L[3]) {
    const int kt = fs_kt(L);
    return (L[0] + kt - 1) / kt * kt;
}
// Bytes of one split B block (144 planes x rows x Lp sites x 8 bytes).
inline size_t fs_block_bytes(const int L[3]) { return (size_t)kFsPlanes * L[1] * L[2] * fs_lp(L) * 8; }
// Dynamic LDS of the fused kernel: the w1 table [nseg][kFacMaxK1][KT + 2] and
// the three root tables (L1 + L2 + L3 entries), complex FP32.
inline size_t fs_dyn_bytes(const int L[3], int kt) {
    const int nseg = (L[0] + kt - 1) / kt;
    return ((size_t)nseg * kFacMaxK1 * (kt + 2) + L[0] + L[1] + L[2]) * 8;
}

hipError_t launch_fs_split(bool bf16, const FsSplitArgs& a, hipStream_t st);
hipError_t launch_fs_diquark(bool bf16, const FsDiquarkArgs& a, hipStream_t st);
// cb: column blocks per workgroup (1 or 2; 2 needs bsplit or kind 0 .. 2 alike, 1 needs bsplit)
hipError_t launch_fs(bool bf16, int KT, int kind, bool bsplit, int cb, const ProjGrid& pg, const FsArgs& a,
                     hipStream_t st);
hipError_t launch_fs_reduce(const FsReduceArgs& a, hipStream_t st);

}  // namespace c3pt
