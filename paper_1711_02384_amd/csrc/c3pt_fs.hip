// Split-precision fused projection: the passes that split propagator slices
// and form the nucleon diquark, the kernel instantiations and the FP64
// reduction of the derivative slots.  The kernel
// itself is in c3pt_fs.h.
#include "c3pt_fs.h"
#include "c3pt_fs_api.h"

namespace c3pt {

// ---------------------------------------------------------------------------
// Propagator slices -> split B blocks.  Plane p' = 48 c + X of block s holds
// B[c][X] = G_s[(bt, c)][(b, c0)] with X = 12 bt + 3 b + c0 (times
// g[bt] g[b] and conjugated for the meson spectator); a block is [row][plane]
// segments of Lp sites (zero beyond L1), four sites per group, so the planes
// of one row lie together.  One thread per (site, plane).
// ---------------------------------------------------------------------------
template <typename T16>
__global__ void __launch_bounds__(256) fs_split_kernel(FsSplitArgs a) {
    const int Lp = a.Lp;
    const long long total = (long long)kFsPlanes * a.rows * Lp * a.n_slices;
    const int L1 = a.L[0];
    const unsigned V3 = (unsigned)(a.L[0] * a.L[1] * a.L[2]);
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int x1 = (int)(idx % Lp);
        long long rest = idx / Lp;
        const int p = (int)(rest % kFsPlanes);
        rest /= kFsPlanes;
        const int row = (int)(rest % a.rows);
        const int sl = (int)(rest / a.rows);
        const int X = p % 48, cs = p / 48;
        const int bt = X / 12, rem = X % 12;
        const float2 v = a.G[sl][(unsigned)((3 * bt + cs) * 12 + rem) * V3 + (unsigned)(min(x1, L1 - 1) + L1 * row)];
        const float sg = a.conj_sign ? (bt < 2 ? 1.f : -1.f) * (rem / 3 < 2 ? 1.f : -1.f) : 1.f;
        const float sy = a.conj_sign ? -sg : sg;
        unsigned hw, lw;
        fs_split2<T16>(x1 < L1 ? f32x2{sg * v.x, sy * v.y} : f32x2{0.f, 0.f}, hw, lw);
        unsigned* dst = (unsigned*)a.out + (((size_t)sl * a.rows + row) * kFsPlanes + p) * (size_t)(Lp / 4) * 8 +
                        (size_t)(x1 >> 2) * 8 + (x1 & 3);
        dst[0] = hw;
        dst[4] = lw;
    }
}

// ---------------------------------------------------------------------------
// Nucleon diquark -> split B blocks ([row][plane] segments, as above).  Block
// (a1', a1), plane p' = 48 c + 3 q + c' with q = 4 a2' + a2:
//   Q[q][c][c'] = sum eps_{abc} eps_{a'b'c'} G1[(a1',a)][(a1,a')] G2[(a2',b)][(a2,b')]
// A workgroup takes R = max(1, 256 / Lp) whole padded rows and one block;
// each thread reads its site's G1 entries of the block once and loops over
// the 16 q, reading G2's (a2', a2) entries.  The nine planes of one q are
// three runs of three consecutive planes, so per q and row the block holds
// three contiguous runs of 3 Lp sites: the split words go through LDS (double
// buffered, one barrier per q) and leave as 16-byte stores that fill whole
// lines.  Items are (row tile, block), block fastest, and consecutive items
// run on one XCD, so the 16 blocks of a tile read G2 from that XCD's L2 and
// each propagator entry comes from HBM once.
// ---------------------------------------------------------------------------
template <typename T16>
__global__ void __launch_bounds__(256) fs_diquark_kernel(FsDiquarkArgs a) {
    const int Lp = a.Lp;
    const int L1 = a.L[0];
    const unsigned V3 = (unsigned)(a.L[0] * a.L[1] * a.L[2]);
    const int R = Lp <= 128 ? 256 / Lp : 1;
    const int nw = gridDim.x, w = blockIdx.x;
    const int full = (nw / 8) * 8;
    const int item = (w < full) ? (w % 8) * (nw / 8) + w / 8 : w;
    const int blk = item % 16;
    const int row0 = (item / 16) * R;
    const int nr = min(R, a.rows - row0);
    const int tid = threadIdx.x;
    const int rl = tid / Lp, x1 = tid % Lp;
    const bool active = rl < nr;
    const int row = row0 + min(rl, nr - 1);
    const int a1p = blk >> 2, a1 = blk & 3;
    const bool ok = active && x1 < L1;
    const unsigned n = (unsigned)(min(x1, L1 - 1) + L1 * row);
    // [buffer][R rows][9 planes][Lp / 4 groups][hi 4 | lo 4], R * Lp <= 256
    __shared__ __attribute__((aligned(16))) unsigned stage[2][9 * 256 * 2];
    C2<float> g1[3][3];
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const float2 x = a.G1[(unsigned)((3 * a1p + u) * 12 + 3 * a1 + v) * V3 + n];
            g1[u][v] = {x.x, x.y};
        }
    unsigned char* out = (unsigned char*)((FsGroup*)a.out + (size_t)blk * kFsPlanes * a.rows * (Lp / 4));
    const int sw = (rl * 9) * (Lp / 4) * 8 + (x1 >> 2) * 8 + (x1 & 3);   // the site's hi word of plane 0
    const int run_units = 3 * Lp / 2;                                      // 16-byte units of one run (3 planes)
    // G2 of the next q is loaded while the current one is formed and written
    auto load_g2 = [&](int q, C2<float> (&g)[3][3]) __attribute__((always_inline)) {
        const int a2p = q >> 2, a2 = q & 3;
#pragma unroll
        for (int u = 0; u < 3; ++u)
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                const float2 y = a.G2[(unsigned)((3 * a2p + u) * 12 + 3 * a2 + v) * V3 + n];
                g[u][v] = {y.x, y.y};
            }
    };
    C2<float> g2[3][3], g2n[3][3];
    load_g2(0, g2);
#pragma unroll 2
    for (int q = 0; q < 16; ++q) {
        unsigned* st = stage[q & 1];
        if (q + 1 < 16) load_g2(q + 1, g2n);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
#pragma unroll
            for (int cp = 0; cp < 3; ++cp) {
                const int d1 = (cp + 1) % 3, d2 = (cp + 2) % 3;
                C2<float> t = cmul(g1[c1][d1], g2[c2][d2]);
                t = cfnma(t, g1[c1][d2], g2[c2][d1]);
                t = cfnma(t, g1[c2][d1], g2[c1][d2]);
                t = cfma(t, g1[c2][d2], g2[c1][d1]);
                unsigned hw, lw;
                fs_split2<T16>(ok ? f32x2{t.x, t.y} : f32x2{0.f, 0.f}, hw, lw);
                if (active) {
                    st[sw + (3 * c + cp) * (Lp / 4) * 8] = hw;
                    st[sw + (3 * c + cp) * (Lp / 4) * 8 + 4] = lw;
                }
            }
        }
        __syncthreads();
        // runs (row, c): planes 48 c + 3 q .. + 2 of the row, contiguous in the block
        for (int e = tid; e < nr * 3 * run_units; e += 256) {
            const int r = e / (3 * run_units), rem = e % (3 * run_units);
            const int c = rem / run_units, k = rem % run_units;
            const u32x4 v = *(const u32x4*)(st + (r * 9 + 3 * c) * (Lp / 4) * 8 + 4 * k);
            unsigned char* dst =
                out + (((size_t)(row0 + r) * kFsPlanes + 48 * c + 3 * q) * (size_t)(Lp / 4)) * 32 + (size_t)k * 16;
            // streaming stores: 2 GB at 48^3, far more than the caches hold
            __builtin_nontemporal_store(v, (u32x4*)dst);
        }
#pragma unroll
        for (int u = 0; u < 3; ++u)
#pragma unroll
            for (int v = 0; v < 3; ++v) g2[u][v] = g2n[u][v];
    }
}

// ---------------------------------------------------------------------------
// FP64 reduction of the insertion's nine slots into its five operators:
//   op 0        = slot 0
//   op 1 + nu   = e^{-i sigma p_nu} slot(1 + 2 nu) - e^{+i sigma p_nu} slot(2 + 2 nu)   (nu = x, y, z)
//   op 4        = slot 7 - slot 8                                                      (nu = t)
// each summed over the chunks in fixed order, times the source factor.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 fs_source_factor(const int (&L)[3], const int (&r)[3], int sigma, int k1, int k2,
                                                    int k3) {
    const long long V3 = (long long)L[0] * L[1] * L[2];
    const long long n = (long long)k1 * r[0] * (L[1] * L[2]) + (long long)k2 * r[1] * (L[0] * L[2]) +
                        (long long)k3 * r[2] * (L[0] * L[1]);
    double s, c;
    sincospi(2.0 * (double)(n % V3) / (double)V3, &s, &c);
    return make_double2(c, -sigma * s);
}

__global__ void __launch_bounds__(256) fs_reduce_kernel(FsReduceArgs a) {
    const long long total = (long long)a.N * a.nt * 5 * a.n_mom_grp * kBlockCols;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(idx % kBlockCols);
        long long rest = idx / kBlockCols;
        const int m = (int)(rest % a.n_mom_grp);
        rest /= a.n_mom_grp;
        const int op = (int)(rest % 5);
        rest /= 5;
        const int j = (int)(rest % a.nt);
        const int i = (int)(rest / a.nt);
        const int cb0 = (i * a.nt + j) * 9;
        auto slot_sum = [&](int s) {
            double sx = 0.0, sy = 0.0;
            for (int ch = 0; ch < a.n_chunks; ++ch) {
                const float2 v =
                    a.partial[(((size_t)ch * a.n_colblocks + cb0 + s) * a.n_mom_grp + m) * kBlockCols + c];
                sx += (double)v.x;
                sy += (double)v.y;
            }
            return make_double2(sx, sy);
        };
        double2 v;
        if (op == 0) {
            v = slot_sum(0);
        } else {
            const int nu = op - 1;
            const double2 jp = slot_sum(1 + 2 * nu), jm = slot_sum(2 + 2 * nu);
            if (nu == 3) {
                v = make_double2(jp.x - jm.x, jp.y - jm.y);
            } else {
                double s, cs;
                sincospi(2.0 * (double)a.ph.k[nu][m] / (double)a.ph.L[nu], &s, &cs);
                const double sg = (double)a.ph.sigma * s;
                // e^{-i sg} jp - e^{+i sg} jm
                v = make_double2(cs * jp.x + sg * jp.y - (cs * jm.x - sg * jm.y),
                                 cs * jp.y - sg * jp.x - (cs * jm.y + sg * jm.x));
            }
        }
        const double2 f = fs_source_factor(a.ph.L, a.ph.r, a.ph.sigma, a.ph.k[0][m], a.ph.k[1][m], a.ph.k[2][m]);
        const size_t G = ((size_t)i * a.n_tau_total + a.j0 + j) * 5 + op;
        a.out[(G * a.n_mom_total + a.m_off + m) * kBlockCols + c] =
            make_double2(f.x * v.x - f.y * v.y, f.x * v.y + f.y * v.x);
    }
}

namespace {
int grid_for(long long total) {
    long long b = (total + 255) / 256;
    return (int)std::min<long long>(std::max<long long>(b, 1), 65536);
}
}  // namespace

hipError_t launch_fs_split(bool bf16, const FsSplitArgs& a, hipStream_t st) {
    const long long total = (long long)kFsPlanes * a.rows * a.Lp * a.n_slices;
    if (bf16)
        hipLaunchKernelGGL(fs_split_kernel<__bf16>, dim3(grid_for(total)), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(fs_split_kernel<_Float16>, dim3(grid_for(total)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_fs_diquark(bool bf16, const FsDiquarkArgs& a, hipStream_t st) {
    const int R = a.Lp <= 128 ? 256 / a.Lp : 1;   // rows per workgroup (the kernel's rule)
    if (a.Lp > 256 || a.Lp % 16 != 0) return hipErrorInvalidValue;
    const long long tiles = ((long long)a.rows + R - 1) / R;
    if (tiles * 16 > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(tiles * 16));
    if (bf16)
        hipLaunchKernelGGL(fs_diquark_kernel<__bf16>, grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(fs_diquark_kernel<_Float16>, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_fs_reduce(const FsReduceArgs& a, hipStream_t st) {
    const long long total = (long long)a.N * a.nt * 5 * a.n_mom_grp * kBlockCols;
    hipLaunchKernelGGL(fs_reduce_kernel, dim3(grid_for(total)), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <typename T16, int KT, int CB>
static hipError_t launch_fs_cb(int kind, bool bsplit, const ProjGrid& pg, const FsArgs& a, hipStream_t st) {
    const dim3 grid(pg.n_share * pg.n_per_share * pg.n_chunks), block(256 * CB);
    const size_t dyn = fs_dyn_bytes(a.L, KT);
    if (kind == 0 && bsplit)
        hipLaunchKernelGGL((fs_kernel<T16, KT, 0, true, CB>), grid, block, dyn, st, pg, a);
    else if (kind == 0)
        hipLaunchKernelGGL((fs_kernel<T16, KT, 0, false, CB>), grid, block, dyn, st, pg, a);
    else if (kind == 1 && bsplit)
        hipLaunchKernelGGL((fs_kernel<T16, KT, 1, true, CB>), grid, block, dyn, st, pg, a);
    else if (kind == 1)
        hipLaunchKernelGGL((fs_kernel<T16, KT, 1, false, CB>), grid, block, dyn, st, pg, a);
    else if (bsplit)
        hipLaunchKernelGGL((fs_kernel<T16, KT, 2, true, CB>), grid, block, dyn, st, pg, a);
    else
        hipLaunchKernelGGL((fs_kernel<T16, KT, 2, false, CB>), grid, block, dyn, st, pg, a);
    return hipGetLastError();
}

template <typename T16, int KT>
static hipError_t launch_fs_t(int kind, bool bsplit, int cb, const ProjGrid& pg, const FsArgs& a, hipStream_t st) {
    if (cb == 3) {
        // three column blocks per workgroup: 16-site tiles, spectators and the
        // local insertion only (the host plans no other)
        if constexpr (KT == 16) {
            const dim3 grid(pg.n_share * pg.n_per_share * pg.n_chunks), block(768);
            const size_t dyn = fs_dyn_bytes(a.L, 16);
            if (kind == 0 && bsplit)
                hipLaunchKernelGGL((fs_kernel<T16, 16, 0, true, 3>), grid, block, dyn, st, pg, a);
            else if (kind == 0)
                hipLaunchKernelGGL((fs_kernel<T16, 16, 0, false, 3>), grid, block, dyn, st, pg, a);
            else if (kind == 1 && !bsplit)
                hipLaunchKernelGGL((fs_kernel<T16, 16, 1, false, 3>), grid, block, dyn, st, pg, a);
            else
                return hipErrorInvalidValue;
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    return cb == 1 ? launch_fs_cb<T16, KT, 1>(kind, bsplit, pg, a, st) : launch_fs_cb<T16, KT, 2>(kind, bsplit, pg, a, st);
}

// 48-site tiles (rows of 48 sites as one tile, a third of the barriers), two
// blocks per workgroup: the spectators and the local insertion
template <typename T16>
static hipError_t launch_fs48(int kind, bool bsplit, int cb, const ProjGrid& pg, const FsArgs& a, hipStream_t st) {
    if (cb != 2) return hipErrorInvalidValue;
    const dim3 grid(pg.n_share * pg.n_per_share * pg.n_chunks), block(512);
    const size_t dyn = fs_dyn_bytes(a.L, 48);
    if (kind == 0 && bsplit)
        hipLaunchKernelGGL((fs_kernel<T16, 48, 0, true, 2>), grid, block, dyn, st, pg, a);
    else if (kind == 0)
        hipLaunchKernelGGL((fs_kernel<T16, 48, 0, false, 2>), grid, block, dyn, st, pg, a);
    else if (kind == 1 && !bsplit)
        hipLaunchKernelGGL((fs_kernel<T16, 48, 1, false, 2>), grid, block, dyn, st, pg, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_fs(bool bf16, int KT, int kind, bool bsplit, int cb, const ProjGrid& pg, const FsArgs& a,
                     hipStream_t st) {
    if (KT == 48) return bf16 ? launch_fs48<__bf16>(kind, bsplit, cb, pg, a, st)
                              : launch_fs48<_Float16>(kind, bsplit, cb, pg, a, st);
    if (bf16)
        return KT == 32 ? launch_fs_t<__bf16, 32>(kind, bsplit, cb, pg, a, st)
                        : launch_fs_t<__bf16, 16>(kind, bsplit, cb, pg, a, st);
    return KT == 32 ? launch_fs_t<_Float16, 32>(kind, bsplit, cb, pg, a, st)
                    : launch_fs_t<_Float16, 16>(kind, bsplit, cb, pg, a, st);
}

}  // namespace c3pt
