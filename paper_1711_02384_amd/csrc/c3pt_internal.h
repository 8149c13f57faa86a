// Internal declarations shared by the host API and the kernels of libc3pt.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace c3pt {

// One column block of the projection GEMM = one 192-component spin-colour group.
constexpr int kBlockCols = 192;
// Largest momentum group handled by one projection launch (FP32 / FP64).
constexpr int kMaxMomGroupF32 = 128;
constexpr int kMaxMomGroupF64 = 32;
constexpr int kMaxMomGroup = 128;
// Largest number of insertion timeslices per launch (pointer tables travel as
// kernel arguments).
constexpr int kMaxTauPerLaunch = 24;
// FP32 partial sums never run over more sites than this before they are
// handed to the FP64 reduction.
constexpr int kMaxSitesPerChunkF32 = 2048;
constexpr int kMaxL = 256;

// Momentum list and phase convention of one momentum group.  Phase tables
// are built for the origin r = 0; the source offset of Sec. 2.1 enters as the
// per-momentum factor exp(-sigma 2 pi i k.r / L) when the sums are written.
struct PhaseSpec {
    int L[3];
    int r[3];          // source position, already reduced into [0, L_j)
    int sigma;         // -1 spectator, +1 insertion
    int n_mom;         // momenta in this group
    uint8_t k[3][kMaxMomGroup];   // components reduced into [0, L_j)
};

// Factored projection (per-direction partial sums).  The phase factorizes,
// exp(i p.x) = w1^(k1 x1) w2^(k2 x2) w3^(k3 x3) with w_j = exp(sigma 2 pi i / L_j),
// so the site sum runs in three stages: over x1 for each distinct k1 (an MFMA
// GEMM), over x2 for each distinct (k1, k2) pair, over x3 for each momentum.
constexpr int kFacTile = 16;          // sites per tile: a segment of one x1 row
constexpr int kFacThreads = 768;      // 12 waves, one 16-column tile each
constexpr int kFacMaxK1 = 8;          // k1 slots: one MFMA row tile (8 x (re, im))
constexpr int kFacMaxPairsF32 = 48;   // distinct (k1, k2) pairs held in LDS
constexpr int kFacMaxPairsF64 = 16;
constexpr int kFacMaxBPerA = 6;       // pairs per k1 slot (per-lane registers of stage 2); a k1
                                      // with more distinct k2 takes several slots
struct FactorPlan {
    int L[3];
    int sigma;
    int n_mom, n1, n12;
    int nbmax;                        // largest number of pairs in one slot
    int k1[kFacMaxK1];                // k1 of slot a (reduced mod L1)
    int bstart[kFacMaxK1 + 1];        // pairs of slot a: b in [bstart[a], bstart[a+1])
    int k2[kFacMaxPairsF32];          // k2 of pair b (reduced mod L2)
    int pair_of_m[kMaxMomGroup];      // pair b of momentum m
    int k3[kMaxMomGroup];             // k3 of momentum m (reduced mod L3)
    int mstart[kFacMaxPairsF32 + 1];  // momenta of pair b: m_of[mstart[b] .. mstart[b+1])
    int m_of[kMaxMomGroup];
};

// One launch of the fused contraction + projection kernel.  Work items are
// (chunk, share, within), chunk outermost, with column block
// cb = colblock(share, within): items that read the same input slice (same
// share) and chunk, and the neighbouring shares of a chunk, are issued to
// the same XCD so that they meet in its L2.
struct ProjGrid {
    int V3;
    int n_mom;         // momenta in this group
    int chunk_sites;   // sites per split-site chunk (multiple of 32)
    int n_chunks;
    int n_colblocks;
    int n_share, n_per_share;
    const void* phase; // phase table of the group (origin r = 0), in the consumer's layout;
                       // factored launches: the FactorPlan of the group
    void* partial;     // [n_chunks][n_colblocks][n_mom][192] partial sums in the accumulator type
                       // (complex float; complex double for complex128 inputs)
    int chunk_planes;  // factored launches: x3 planes per chunk (chunk_sites unused)
    int fac_acc;       // factored launches: sum a chunk's planes in registers
};

// Producer arguments -------------------------------------------------------
struct MesonSpecArgs {
    int L[3];
    const void* G;     // [144][V3]
    const void* eta;   // [N][12][V3]
};

struct BaryonSpecArgs {
    int L[3];
    const void* G1;
    const void* G2;
    const void* eta;
};

struct InsertionArgs {
    int L[3];
    int n_tau;         // timeslices in this launch
    int n_ops;         // 1 or 5
    int n_noise;
    int op_lo, op_cnt; // operators covered by this launch's work items: [op_lo, op_lo + op_cnt)
    const void* G[kMaxTauPerLaunch];     // G(tau)
    const void* Gn[kMaxTauPerLaunch];    // G(tau+1)  (derivative ops only)
    const void* Gp[kMaxTauPerLaunch];    // G(tau-1)
    const void* s[kMaxTauPerLaunch];     // s(tau) [N][12][V3]
    const void* U[kMaxTauPerLaunch];     // U(tau) [4][3][3][V3]
    const void* Up[kMaxTauPerLaunch];    // U(tau-1)
};

// One job of a batch (device copy): a spectator or an insertion call.
struct BatchJob {
    int kind;          // 0 meson spectator, 1 baryon spectator, 2 insertion
    int V3, L[3], r[3];
    int sigma;
    int n_noise, n_tau, n_ops;
    int n_colblocks, n_chunks, chunk_sites;
    int group_cols;    // 192 or 3072 output columns per group
    int n_mom;         // momenta (at most 128)
    const int* k;      // device [n_mom][3] momentum list (signed; reduced per job)
    // Output group of job-local group g: (g / out_inner) * out_stride + out_off + g % out_inner
    // (a job may cover a block of noise vectors or timeslices of a larger output).
    int out_inner, out_stride, out_off;
    const void* G;     // spectator propagator (baryon: G1)
    const void* G2;    // baryon: G2
    const void* eta;   // spectator noise
    const void* const* tau_ptrs;   // insertion: device table [n_tau][6] = G, G(+1), G(-1), s, U, U(-1)
    const void* phase; // phase table (origin r = 0) for (L, sigma, momenta, layout)
    void* partial;     // [n_chunks][n_colblocks][n_mom][192] (complex float)
    double2* out;      // output in the layout of the single call
};

// A projection launch over the items of several jobs of one kind (factored:
// one workgroup per item; dense: persistent workgroups taking items from the
// queue whose head is `counter`).
struct BatchGrid {
    const BatchJob* jobs;
    const int4* items;     // (job, column block, chunk, 0) in issue order
    int n_items;
    int* counter;          // work-queue head, zeroed by the batch's reset kernel
};

// Batched reduction: one output element per thread over all jobs of a group.
struct BatchReduceArgs {
    const BatchJob* jobs;
    const long long* out_offset;   // prefix sums of the jobs' output elements (n_jobs + 1)
    int n_jobs;
};

// Reduction of the split-site partial sums: output[G][m][c], c < group_cols,
// with output group G = (g / inner) * outer_stride + off + g % inner for the
// launch-local group g (this places a subset of insertion timeslices).
struct ReduceArgs {
    const void* partial;
    int f64;           // partials are complex double (else complex float)
    double2* out;
    PhaseSpec ph;      // momenta of the group, source position and sign (for the source factor)
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
    const double2* I;     // [N][n_tau_in][n_ops][n_q][192]
    const double* w;      // device [N]
    const int* pairs;     // device [n_pairs][2] or null (all pairs)
    double2* out;         // [n_pairs][n_tau][n_sel][spin][64]
    int n_noise, n_p, n_q, n_tau, n_ops, op_begin, n_sel, spin, n_pairs;
    // timeslice window of the insertion: output tau reads insertion slice
    // tau0 + tau of n_tau_in (0: the insertion holds exactly the n_tau slices)
    int tau0 = 0, n_tau_in = 0;
};

// Arithmetic of a projection launch.
constexpr int kModeF64 = 0;         // complex128 inputs, FP64 MFMA
constexpr int kModeF32 = 1;         // complex64 inputs, FP32 MFMA
constexpr int kModeSplitBF16 = 2;   // complex64 inputs, hi+lo BF16 MFMA, FP32 accumulation
constexpr int kModeSplitF16 = 3;    // complex64 inputs, hi+lo FP16 MFMA, FP32 accumulation
// Chunk sizes are multiples of the largest site tile of any variant.
constexpr int kSiteTile = 32;
// Momentum-tile classes (8 momenta per 16-row MFMA tile): mt <= 4, 8, 12, 16.
constexpr int kMtClasses = 4;
__host__ __device__ inline int mt_class(int mt) { return mt <= 4 ? 0 : mt <= 8 ? 1 : mt <= 12 ? 2 : 3; }
// Compiled (site tile, row split) variants per class; FP64 has one (class 0).
constexpr int kVariantsPerClass[kMtClasses] = {2, 3, 3, 2};

// Launchers (c3pt_proj_*.hip, c3pt_combine.hip). They return the launch status.
hipError_t launch_spectator_meson(int mode, int mt, int variant, const ProjGrid& pg, const MesonSpecArgs& a,
                                  hipStream_t st);
hipError_t launch_spectator_baryon(int mode, int mt, int variant, const ProjGrid& pg, const BaryonSpecArgs& a,
                                   hipStream_t st);
hipError_t launch_insertion(int mode, int mt, int variant, const ProjGrid& pg, const InsertionArgs& a,
                            hipStream_t st);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st);
// Factored projection launches (f64: complex128 inputs, FP64 MFMA; else FP32).
// acc: sum a chunk's x3 planes in registers (else in the partial sums, in place).
hipError_t launch_fac_meson(bool f64, bool acc, const ProjGrid& pg, const MesonSpecArgs& a, hipStream_t st);
hipError_t launch_fac_baryon(bool f64, bool acc, const ProjGrid& pg, const BaryonSpecArgs& a, hipStream_t st);
// ops: 1 local operator only, 2 derivative operators only (a.op_lo / a.op_cnt select them)
hipError_t launch_fac_insertion(bool f64, bool acc, int ops, const ProjGrid& pg, const InsertionArgs& a,
                                hipStream_t st);
// Factored launches (FP32) over batch items, one workgroup per item.  With
// bg == nullptr only the occupancy (workgroups per CU) is returned.  variant
// bits: kBatchFacKT32 takes 32-site tiles, honoured only by producers whose
// registers allow them (batch_fac_allows32) and passed by the caller only when
// every job of the launch has L1 % 32 == 0; kBatchFacWide is read by the
// planner, which then puts about 4096 instead of 2048 sites in a chunk
// (batch_fac_chunk_planes).
constexpr int kBatchFacKT32 = 1, kBatchFacWide = 2, kBatchFacVariants = 4;
// variant slot ("mode" of c3pt_set_variant) that holds these choices per producer kind
constexpr int kModeBatchFacVariants = 6;
// queue kinds: 0 meson spectator, 1 baryon spectator, 2 insertion local operator,
// 3 insertion derivative operators
inline bool batch_fac_allows32(int queue_kind) { return queue_kind == 0 || queue_kind == 2; }
inline int batch_fac_chunk_planes(const int L[3], int variant) {
    const int sites = (variant & kBatchFacWide) ? 4096 : 2048;
    const int p = sites / (L[0] * L[1]);
    return p < 1 ? 1 : (p > L[2] ? L[2] : p);
}
int batch_fac_meson(int variant, const BatchGrid* bg, hipStream_t st, hipError_t* err);
int batch_fac_baryon(int variant, const BatchGrid* bg, hipStream_t st, hipError_t* err);
int batch_fac_insertion(int variant, int ops, const BatchGrid* bg, hipStream_t st, hipError_t* err);
// Factor plan of a momentum list for extents L and sign sigma (FP32 limits);
// false if the list needs more distinct k1 / (k1, k2) than the kernel holds.
bool api_factor_plan(const int L[3], int sigma, const int* k, int n_mom, FactorPlan* plan);
// Dense persistent batch launch of one producer kind; with bg == nullptr only the
// occupancy (workgroups per CU) of the variant is returned.
int batch_meson(int mode, int mt, int variant, const BatchGrid* bg, int n_wg, hipStream_t st, hipError_t* err);
int batch_baryon(int mode, int mt, int variant, const BatchGrid* bg, int n_wg, hipStream_t st, hipError_t* err);
int batch_insertion(int mode, int mt, int variant, const BatchGrid* bg, int n_wg, hipStream_t st, hipError_t* err);
hipError_t launch_batch_reduce(const BatchReduceArgs& a, long long total, hipStream_t st);
hipError_t launch_reset(int* counters, int n, hipStream_t st);
// Phase tables (c3pt_phase.hip).  Native layout: [Vpad][8*mtmax] complex
// (double for mode kModeF64, float for kModeF32).  Split layout:
// [Vpad/16][hi, lo][mtmax][64 lanes][8] 16-bit values in MFMA A-operand order.
// Vpad = V3 rounded up to 32; padding sites and rows hold zeros.
size_t phase_table_bytes(int mode, int V3, int mtmax);
hipError_t launch_phase_table(int mode, const PhaseSpec& ph, int V3, int mtmax, void* out, hipStream_t st);
hipError_t launch_combine(const CombineArgs& a, hipStream_t st);

}  // namespace c3pt
