/*
 * c3pt.h -- C ABI of the spin-open three-point contraction library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library computes the hot path of the factorized stochastic three-point
 * function of Bali et al., "Baryonic and mesonic 3-point functions with open
 * spin indices" (Lattice 2017):
 *
 *   spectator part, Eq. (9)      c3pt_spectator_meson / c3pt_spectator_baryon
 *   insertion part, Eq. (10)     c3pt_insertion
 *   noise-averaged product of the two parts (Eq. (5) in Eq. (8))   c3pt_combine
 *   forward + backward diagrams, time-partitioned noise (Sec. 2.3)  c3pt_two_sink_meson
 *   Gamma channels of the spin-open data (Eq. (1), Sec. 3)  c3pt_gamma_meson / c3pt_gamma_nucleon
 *   gauge-covariant smearing of the inputs (Sec. 2.1, Sec. 3)  c3pt_smear
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Complex numbers are interleaved (re, im) pairs.  Inputs are complex64
 *    (float2) or complex128 (double2) as selected by c3pt_geom.dtype; every
 *    output is complex128.
 *  - Spin-colour index A = 3*spin + colour (spin 0..3, colour 0..2).  Gamma
 *    matrices are in the DeGrand-Rossi basis, so gamma5 = diag(1, 1, -1, -1).
 *  - Spatial site n = x1 + L1*(x2 + L2*x3).  Every field is given per timeslice,
 *    structure-of-arrays with the site index fastest:
 *        propagator slice   G[A_row][A_col][site]   (12*12*V3 complex),
 *                            row = field point, column = source point;
 *        noise eta / stochastic solution s   v[noise][A][site]  (N*12*V3),
 *        gauge links        U[mu][c][d][site]  (4*3*3*V3), mu = x, y, z, t,
 *                            U_mu(x) on the link x -> x + mu.
 *  - Momenta: host array k[n_mom][3] of integers; the phase of site x is
 *        exp(sigma * 2 pi i * sum_j k_j (x_j - r_j) / L_j)
 *    with sigma = -1 for spectators (Eq. (9)) and +1 for insertions (Eq. (10)),
 *    and r the spatial source position (Sec. 2.1).  Components may be any
 *    integers; they are reduced modulo L_j.
 *
 * Memory and execution
 * --------------------
 *  - All field and output pointers are DEVICE pointers owned by the caller.
 *    Pointer tables (G_t, s_t, U_t), k, taus, w and pairs are HOST arrays read
 *    during the call only.
 *  - Calls are asynchronous on the given HIP stream (NULL = the null stream):
 *    results are valid once the stream has been synchronized.  Scratch space
 *    (split-site partial sums) is owned by the library, one buffer per stream,
 *    grown on demand; growing synchronizes that stream.  Calls on one stream
 *    are ordered; calls on different streams do not share scratch space.
 *  - Results are deterministic: no floating-point atomics; split-site partial
 *    sums are reduced in a fixed order in FP64.
 *
 * Errors
 * ------
 *  Every entry point returns C3PT_OK (0) or a negative status.  Arguments are
 *  validated before anything is enqueued: on error nothing is launched and the
 *  output buffer is untouched.  c3pt_last_error() gives a message for the last
 *  failing call on the calling thread.  No C++ exception crosses this ABI.
 */
#ifndef C3PT_H
#define C3PT_H

#ifdef __cplusplus
extern "C" {
#endif

#define C3PT_OK            0
#define C3PT_EINVAL       (-1)   /* bad extents, NULL pointer, index out of range  */
#define C3PT_ENOMEM       (-2)   /* scratch allocation failed                      */
#define C3PT_EDEVICE      (-3)   /* a HIP call failed                              */
#define C3PT_EUNSUPPORTED (-4)   /* valid request this build cannot execute        */

#define C3PT_C64   0              /* complex64 inputs (FP32 contractions)  */
#define C3PT_C128  1              /* complex128 inputs (FP64 throughout)   */

#define C3PT_PROJ_NATIVE      0   /* projection in the input precision (FP32 or FP64 MFMA)     */
#define C3PT_PROJ_SPLIT_F16   1   /* complex64 only: hi+lo FP16 operands, FP32 MFMA accumulate */
#define C3PT_PROJ_SPLIT_BF16  2   /* complex64 only: hi+lo BF16 operands, FP32 MFMA accumulate */
#define C3PT_PROJ_FACTORED    3   /* per-direction partial sums (exp(ip.x) = product over x1, x2,
                                     x3), stage over x1 on FP32 / FP64 MFMA; momentum groups needing
                                     more than 8 distinct k1 or 48 (FP64: 24) distinct (k1, k2)
                                     run on the NATIVE kernel                                    */

#define C3PT_PROJ_FACTORED_F16  4   /* complex64 only: factored projection with the colour
                                       contraction folded into its x1 stage, which runs on
                                       hi+lo FP16 MFMA with FP32 accumulation (B operand split
                                       once per call); spectators and n_ops 1 / 5 insertions,
                                       momentum lists that factor (else C3PT_EUNSUPPORTED)   */
#define C3PT_PROJ_FACTORED_BF16 5   /* the same with hi+lo BF16 operands                        */

#define C3PT_MAX_MOM   256        /* largest momentum list per call        */
#define C3PT_MAX_L     256        /* largest spatial extent per direction  */

typedef struct c3pt_geom {
    int   L[3];     /* spatial extents L1, L2, L3 (each 1..C3PT_MAX_L)           */
    int   T;        /* temporal extent (>= 1); time neighbours wrap modulo T     */
    int   r[3];     /* spatial source position, the origin of the phases         */
    int   dtype;    /* C3PT_C64 or C3PT_C128                                     */
    int   proj;     /* C3PT_PROJ_*                                               */
    void* stream;   /* hipStream_t the work is enqueued on; NULL = null stream   */
} c3pt_geom;

/*
 * Meson spectator part, Eq. (9):
 *   S_i(p')[b'][a'][a][c] = sum_x' exp(-i p'.(x'-r)) sum_c' [gamma5 eta_i(x')]^{b'}_{c'}
 *                           [gamma5 G(x',r)^dag gamma5]^{a' a}_{c' c}
 * i.e. g[b'] g[a'] g[a] sum_c' eta_i[(b',c')] conj(G[(a',c')][(a,c)]) per site.
 *   G_tf : device, propagator slice at the sink timeslice, 144*V3 complex.
 *   eta  : device, n_noise noise vectors on the sink timeslice, n_noise*12*V3.
 *   out  : device, complex128 [n_noise][n_mom][192], spin order (b', a', a, c).
 */
int c3pt_spectator_meson(const c3pt_geom* geom, const void* G_tf, const void* eta, int n_noise,
                         const int* k, int n_mom, void* out);

/*
 * Nucleon-type spectator with epsilon-tensor colour contraction.  The paper
 * times a baryon measurement without printing its formula; this is the
 * reading in which the two spectator quarks run forward from the source
 * (G1, G2) and the active quark leaves the sink on the stochastic line exactly
 * as in Eq. (8):
 *   S_i(p')[a1'][a1][a2'][a2][b'][c'] = sum_x' exp(-i p'.(x'-r)) g[b'] sum_c eta_i[(b',c)]
 *        sum eps_{abc} eps_{a'b'c'} G1[(a1',a)][(a1,a')] G2[(a2',b)][(a2,b')]
 *   G1_tf, G2_tf : device propagator slices at the sink timeslice.
 *   out          : device complex128 [n_noise][n_mom][3072],
 *                  order (a1', a1, a2', a2, b', c').
 */
int c3pt_spectator_baryon(const c3pt_geom* geom, const void* G1_tf, const void* G2_tf,
                          const void* eta, int n_noise, const int* k, int n_mom, void* out);

/*
 * Insertion part, Eq. (10), at every timeslice tau in taus[0..n_tau):
 *   I_i(q,tau)[op][at][bt][b][c] = sum_y exp(+i q.(y-r)) g[at]
 *        sum_c' conj(s_i(y)[(at,c')]) (O_op G)(y)[(bt,c')][(b,c)]
 * with O_0 = 1 (all 16 Gamma stay open in (at, bt)) and, when n_ops >= 5,
 * O_{1+nu} = D_nu, nu = x, y, z, t (the local derivatives of Sec. 2.1):
 *   (D_nu G)(y) = 1/2 [U_nu(y) G(y+nu) - U_nu(y-nu)^dag G(y-nu)],
 * spatial neighbours periodic in L_j, time neighbours taken modulo T.
 * With n_ops == 9, ops 5+nu are the symmetrized derivative
 *   <->D_nu = 1/2 (->D_nu - <-D_nu),
 * where the left derivative acts on the insertion's antiquark; in the
 * factorized form it is D_nu applied to s: op 5+nu = 1/2 (op 1+nu - I[s -> D_nu s]).
 * With n_ops == 21, ops 5 + 4 rho + nu are the two-derivative operators
 * D_nu D_rho (D_rho applied first): D_rho G is formed on tau-1 .. tau+1 by a
 * stencil into the library's per-stream scratch, then D_nu of it is contracted.
 * With n_ops == 37, ops 21 + 4 mu + nu are in addition the symmetrized
 *   <->D_mu <->D_nu = 1/4 (->D_mu ->D_nu - ->D_mu <-D_nu - <-D_mu ->D_nu + <-D_mu <-D_nu),
 * the left derivatives acting on the antiquark (D applied to s, <-D_mu first).
 * n_ops == 9, 21 and 37 run on the factored projection only
 * (C3PT_PROJ_FACTORED and a momentum list it factors; C3PT_EUNSUPPORTED
 * otherwise).
 *   G_t : host array of T device pointers (slice t of the propagator, or NULL
 *         where not needed).  Needed: every tau; with n_ops >= 5 also tau+-1;
 *         with n_ops >= 21 also tau+-2.
 *   s_t : host array of T device pointers to [n_noise][12][V3]; needed at every
 *         tau; with n_ops == 9 also at tau+-1; with n_ops == 37 at tau+-1, tau+-2.
 *   U_t : host array of T device pointers to [4][3][3][V3], or NULL when
 *         n_ops == 1.  With n_ops >= 5 needed at every tau and tau-1; with
 *         n_ops >= 21 also tau+1 and tau-2.
 *   out : device complex128 [n_noise][n_tau][n_ops][n_mom][192],
 *         order (at, bt, b, c).
 */
int c3pt_insertion(const c3pt_geom* geom, const void* const* G_t, const void* const* s_t,
                   int n_noise, const int* taus, int n_tau, const void* const* U_t, int n_ops,
                   const int* k, int n_mom, void* out);

/*
 * c3pt_insertion without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, layouts and results as c3pt_insertion,
 * restricted to n_ops 1 or 5, geom->proj == C3PT_PROJ_FACTORED and momentum
 * lists the factored projection takes (else C3PT_EUNSUPPORTED).
 * Its FP32 (FP64) partial sums and the factor plan live in one fixed device
 * array of C3PT_NOALLOC_SCRATCH_BYTES, which each GPU the library runs on
 * holds from the first call until the process ends; the call runs its
 * timeslices in launch groups whose partial sums fit the array.  A request
 * whose single timeslice needs more is rejected with C3PT_EINVAL before
 * anything is enqueued (its message gives both sizes).  The call enqueues
 * only kernels: no hipMalloc, hipFree, host copy or event.
 * Every call on one GPU shares that GPU's array, whose contents are what the
 * last call left: calls that overlap on one GPU (different streams, or host
 * threads) race and must be ordered by the caller.  c3pt_noalloc_scratch_bytes()
 * returns the array's size.
 */
#define C3PT_NOALLOC_SCRATCH_BYTES (128u << 20)
unsigned long long c3pt_noalloc_scratch_bytes(void);
int c3pt_insertion_noalloc(const c3pt_geom* geom, const void* const* G_t, const void* const* s_t,
                           int n_noise, const int* taus, int n_tau, const void* const* U_t, int n_ops,
                           const int* k, int n_mom, void* out);

/*
 * Noise-weighted product of spectator and insertion (Eq. (5) inserted into
 * Eq. (8)), summing the source colour shared by the two parts (the delta of
 * Eq. (1)):
 *   C[pair][tau][op - op_begin][s][t] = sum_i w_i sum_c S_i(p'_pair)[s][c] I_i(q_pair, tau)[op][t][c]
 *   spec      : device complex128 [n_noise][n_p][spec_spin*3] (spec_spin 64 or 1024),
 *               the output of a spectator call.
 *   ins       : device complex128 [n_noise][n_tau][n_ops][n_q][192], an insertion output.
 *   w         : host [n_noise] weights, or NULL for 1/n_noise.
 *   pairs     : host [n_pairs][2] (p' index, q index), or NULL for all n_p*n_q pairs
 *               in the order p'*n_q + q (then n_pairs must be n_p*n_q).
 *   op_begin, op_end : the half-open range of insertion operators combined.
 *   out       : device complex128 [n_pairs][n_tau][op_end-op_begin][spec_spin][64].
 * Computed entirely in FP64.
 */
int c3pt_combine(const void* spec, int spec_spin, const void* ins, int n_noise, int n_p, int n_q,
                 int n_tau, int n_ops, int op_begin, int op_end, const double* w, const int* pairs,
                 int n_pairs, void* out, void* stream);

/*
 * One meson measurement with time-partitioned noise, forward and backward
 * diagrams together (Sec. 2.3, Fig. 6): the noise vectors are zero except on
 * the two sink timeslices t_fwd = x'_4 and t_bwd = x''_4 on either side of the
 * source timeslice t_src = r_4, and one stochastic solution per noise vector
 * serves both diagrams.  The call runs
 *   spectators : c3pt_spectator_meson at t_fwd (G_fwd, eta_fwd) and at t_bwd
 *                (G_bwd, eta_bwd);
 *   insertion  : c3pt_insertion at tau = t_fwd, t_fwd+1, ..., t_bwd (modulo T,
 *                n_span = n_fwd + n_bwd - 1 slices);
 *   combines   : forward  = S(t_fwd) x I(tau), tau = t_fwd .. t_src (n_fwd slices),
 *                backward = S(t_bwd) x I(tau), tau = t_src .. t_bwd (n_bwd slices),
 *                each as c3pt_combine over all n_ops operators;
 * with n_fwd = ((t_src - t_fwd) mod T) + 1 and n_bwd = ((t_bwd - t_src) mod T) + 1,
 * n_fwd + n_bwd - 1 <= T.  The source timeslice is in both windows.
 *   G_fwd, G_bwd     : device propagator slices at the two sinks [12][12][V3].
 *   eta_fwd, eta_bwd : device noise slices at the two sinks [n_noise][12][V3].
 *   G_t, s_t, U_t, n_ops, k, n_mom : as for c3pt_insertion, needed on the span.
 *   w, pairs, n_pairs : as for c3pt_combine with n_p = n_q = n_mom.
 *   spec    : device complex128 [2][n_noise][n_mom][192], forward then backward
 *             spectator (order as c3pt_spectator_meson).
 *   ins     : device complex128 [n_noise][n_span][n_ops][n_mom][192].
 *   out_fwd : device complex128 [n_pairs][n_fwd][n_ops][64][64].
 *   out_bwd : device complex128 [n_pairs][n_bwd][n_ops][64][64].
 * Every argument is checked before anything is enqueued.
 */
int c3pt_two_sink_meson(const c3pt_geom* geom, const void* G_fwd, const void* eta_fwd, int t_fwd,
                        const void* G_bwd, const void* eta_bwd, int t_bwd, int t_src, int n_noise,
                        const void* const* G_t, const void* const* s_t, const void* const* U_t, int n_ops,
                        const int* k, int n_mom, const double* w, const int* pairs, int n_pairs, void* spec,
                        void* ins, void* out_fwd, void* out_bwd);

/*
 * Analysis stage: Gamma channels of the spin-open meson data.  The trace of
 * Eq. (1) for any Gamma_snk, Gamma_ins and source matrix follows from the
 * combine output by contracting its open spins (Sec. 1, Sec. 3):
 *   out[blk][i][j][l] = sum Gsnk_i[a'][b'] Gins_j[at][bt] Gsrc_l[b][a] C[blk][b'][a'][a][at][bt][b]
 *   C     : device complex128 [n_blk][64][64], rows (b', a', a), columns
 *           (at, bt, b): any number of blocks of c3pt_combine's meson output
 *           (pair, timeslice, operator).  For a derivative operator D_nu,
 *           Gins = gamma_mu gives gamma_mu D_nu.
 *   g_snk, g_ins, g_src : host complex128 [n][4][4] (interleaved re, im; row
 *           index first), 1 <= n <= 16; NULL selects the 16 Gamma_n =
 *           g1^b0 g2^b1 g3^b2 g4^b3 (n = b0 + 2 b1 + 4 b2 + 8 b3) for g_snk and
 *           g_ins and the creation matrices gamma4 Gamma_n^dag gamma4 of
 *           Eq. (3) for g_src (then the count must be 16).
 *   out   : device complex128 [n_blk][n_snk][n_ins][n_src].
 * FP64 throughout.
 */
int c3pt_gamma_meson(const void* C, int n_blk, const double* g_snk, int n_snk, const double* g_ins, int n_ins,
                     const double* g_src, int n_src, void* out, void* stream);

#define C3PT_PROTON_D  0   /* current on the d quark: spectators (G1, G2) = (u, u)  */
#define C3PT_PROTON_U  1   /* current on a u quark: spectators (G1, G2) = (u, d)    */

/*
 * Analysis stage for the nucleon data (the paper times a baryon measurement,
 * Sec. 3, without printing its contraction; the reading used here): proton
 * chi_g = eps_abc (u_a^T A d_b) u_c^g at the sink, chibar = chi^dag gamma4 =
 * eps_abc ubar_c (dbar_b Abar ubar_a^T) at the source, current J_j =
 * qbar Gins_j q; connected Wick contractions with the proton's two (d
 * current) or four (u current) pairings of the identical u quarks:
 *   out[blk][p][j] = tr[P_p G_j],  G_j[g][d] = <chi_g(x') J_j(y) chibar_d(r)>,
 * evaluated from the combine's nucleon output of the matching spectator pair.
 *   C       : device complex128 [n_blk][1024][64] (rows a1', a1, a2', a2, b';
 *             columns at, bt, b), blocks of c3pt_combine's nucleon output.
 *   channel : C3PT_PROTON_D or C3PT_PROTON_U.
 *   A, Abar : host complex128 [4][4] or NULL for A = C gamma5 with
 *             C = gamma2 gamma4 and Abar = gamma4 A^dag gamma4.
 *   P       : host complex128 [n_proj][4][4] (1 <= n_proj <= 16), or NULL for
 *             (1 + gamma4)/2 and (1 - gamma4)/2 (n_proj = 2).
 *   g_ins   : host complex128 [n_ins][4][4] (1 <= n_ins <= 16) or NULL for the
 *             16 Gamma_n (n_ins = 16).
 *   out     : device complex128 [n_blk][n_proj][n_ins].
 * FP64 throughout.  Only rows of C with a non-zero weight are read.
 */
int c3pt_gamma_nucleon(const void* C, int n_blk, int channel, const double* A, const double* Abar,
                       const double* P, int n_proj, const double* g_ins, int n_ins, void* out, void* stream);

/*
 * Gauge-covariant quark smearing of colour vectors on one timeslice, n_iter
 * steps of (Wuppertal form; the paper smears the spectator's propagators at
 * source and sink, Sec. 3, and lets the operators contain smearing, Sec. 2.1,
 * without giving the kernel or its parameters):
 *   psi'(x) = [psi(x) + kappa sum_{j=x,y,z} (U_j(x) psi(x+j) + U_j(x-j)^dag psi(x-j))] / (1 + 6 kappa)
 * with periodic spatial neighbours.
 *   in, out : device fields [n_outer][3][n_inner][V3] (c3pt_geom.dtype), colour
 *             the second index: a propagator slice [12][12][V3] smeared on its
 *             row (field) index is n_outer = 4, n_inner = 12; noise or solution
 *             vectors [N][12][V3] are n_outer = 4 N, n_inner = 1.  in == out is
 *             allowed; otherwise the two must not overlap.
 *   U       : device links of the timeslice [4][3][3][V3] (the time links unused).
 *   kappa   : hopping weight, 0 <= kappa < 1e6;  n_iter >= 0 (0 copies).
 * Uses this stream's scratch for the intermediate steps (one field).
 */
int c3pt_smear(const c3pt_geom* geom, const void* in, void* out, int n_outer, int n_inner, const void* U,
               double kappa, int n_iter);

/* Static description of a status code. */
const char* c3pt_strerror(int status);

/* Message of the last failing call on this thread ("" if none). */
const char* c3pt_last_error(void);

/* Library ABI version (major*100 + minor). */
int c3pt_version(void);

/* Bytes of scratch currently held for `stream` (0 if none). */
unsigned long long c3pt_scratch_bytes(void* stream);

/* Release the scratch buffers of every stream and the cached phase tables
 * (synchronizes the devices involved).  Phase tables (exp(i p.x) per site and
 * momentum, in the layout the kernels read) are built on first use of a
 * (geometry, source, sign, momentum group, arithmetic) and cached, up to 2 GiB
 * per process. */
int c3pt_release_scratch(void);

/*
 * Kernel timing.  While enabled, every kernel the library launches is
 * bracketed by a pair of HIP events on its stream.  c3pt_profile_read()
 * synchronizes those events, folds them into per-kernel statistics and copies
 * up to `max` entries into `stats` (returns the number of kernels seen, or a
 * negative status).  `reset` != 0 clears the statistics after copying.
 * Names: "proj_spectator_meson", "proj_spectator_baryon", "proj_insertion",
 * "reduce", "combine".
 */
/*
 * Kernel variants (tile shapes) of the fused contraction + projection, for
 * the autotuner.  kind: 0 meson spectator, 1 baryon spectator, 2 insertion.
 * mode: 0 FP64 (complex128 inputs), 1 FP32, 2 split BF16, 3 split FP16;
 * mode 4 selects the form of the factored projection (C3PT_PROJ_FACTORED):
 * variant 0 writes every x3 plane's sums as a chunk of its own, variant 1
 * sums chunks of planes in registers first.  Mode 5 selects the form of the
 * split-precision fused projection (C3PT_PROJ_FACTORED_F16 / _BF16):
 * variant 0 splits each propagator tile into hi + lo parts in the kernel and
 * runs two column blocks per workgroup, variant 1 splits the call's slices
 * once in a pass before it, variant 2 does that and runs one column block per
 * workgroup, variant 3 splits in the kernel with one column block per
 * workgroup, variant 4 splits in the kernel with three column blocks per
 * workgroup (16-site tiles, spectators and the local insertion; factor plans
 * with at most five (k1, k2) pairs per k1 slot; when N is not a multiple of
 * three the last N % 3 noise vectors run as a second, two-block launch;
 * elsewhere it runs as variant 0), variant 5 takes rows of 48 sites as one
 * tile when L1 = 48 (spectators and the local insertion; elsewhere as 0).
 * The nucleon spectator always forms its diquark in a pass (variants 0 and
 * 1, and 2 and 3, are the same for it).  Mode 6 selects
 * the factored kernels of batches and of the server (read when a batch is
 * created and when the server plans a step), as two bits: 1 takes 32-site
 * tiles for jobs with L1 % 32 == 0 (meson spectator and local insertion; the
 * other producers keep 16), 2 makes chunks of about 4096 instead of 2048
 * sites.
 * mt_class: momentum groups of up to 32, 64, 96, 128 momenta (0..3).
 * c3pt_variant_count returns the number of compiled variants (0 if none);
 * c3pt_set_variant selects one for later calls (process-wide);
 * c3pt_get_variant returns the current choice or a negative status.
 * Every variant computes the same result up to FP32 rounding order.
 */
/*
 * Extent checks.  Before a call enqueues anything, the bytes each of its
 * kernels will index in every library-sized buffer (partial sums, phase
 * tables, split propagator blocks, the fixed scratch) are compared with the
 * bytes allocated for it; a mismatch fails the call with C3PT_EINVAL and a
 * message naming the buffer.  c3pt_debug_scale_allocations(s) multiplies
 * every allocated size in these comparisons by s (0 < s; 1 restores them): a
 * test hook that plants an under-allocation without touching the device.
 * Builds with C3PT_SYNC_LAUNCHES defined (build.py --debug) also wait for
 * every launch and report a device fault at the launch that caused it.
 */
void c3pt_debug_scale_allocations(double scale);

int c3pt_variant_count(int kind, int mode, int mt_class);
int c3pt_set_variant(int kind, int mode, int mt_class, int variant);
int c3pt_get_variant(int kind, int mode, int mt_class);

typedef struct c3pt_kernel_stat {
    char      name[48];
    long long count;
    double    total_ms;
    double    min_ms;
    double    max_ms;
} c3pt_kernel_stat;

int c3pt_profile_enable(int on);
int c3pt_profile_read(c3pt_kernel_stat* stats, int max, int reset);

/*
 * Batches.  A measurement evaluates the spectator and insertion parts for
 * many source positions, sink times and lattices (Sec. 2.2-2.3: the paper
 * spreads them over MPI ranks); a batch runs many such calls as one unit of
 * work on one GPU.  c3pt_batch_create validates every job, builds the phase
 * tables and work queues and records the whole schedule into one HIP graph;
 * c3pt_batch_run replays it.  The projection work of all jobs of one kind is
 * one launch over a list of (job, column block, site chunk) items (factored:
 * one workgroup per item, handed out in order as CUs free up; dense: a
 * persistent kernel whose workgroups take items from a queue), so lattices of
 * different sizes share the chip until the last item.  A job's sites are
 * summed in FP32 chunks (at most 2048 sites, or whole x3 planes of about 2048
 * or 4096 sites for the factored kernels, fixed by its own extents and the
 * tuned variant) and the chunks in FP64 in a
 * fixed order, so its output does not depend on the other jobs of the batch
 * or on the schedule: a job gives bit-identical results alone or in any mix
 * (with the same kernel variant).  Against the single calls, which split
 * sites differently to fill the chip, results agree to FP32 rounding order.
 *
 *   kind         C3PT_JOB_SPECTATOR_MESON / _BARYON / C3PT_JOB_INSERTION
 *   L, T, r      extents and source position, as in c3pt_geom.  Batch inputs
 *                are complex64 (the FP32 or split-precision projection
 *                selected by `proj` of c3pt_batch_create).
 *   n_noise      noise vectors of the job.
 *   G, G2, eta   spectator inputs as for c3pt_spectator_meson (G) or
 *                c3pt_spectator_baryon (G = G1, G2); device pointers.
 *   G_t, s_t, U_t, taus, n_tau, n_ops   insertion inputs as for c3pt_insertion
 *                (host pointer tables, read during c3pt_batch_create only; the
 *                device buffers they name are read on every run).
 *   out          device complex128 output in the layout of the single call.
 *
 * Combines take the outputs of a spectator job and an insertion job of the
 * same batch (same n_noise) and run after every projection, as c3pt_combine
 * with the batch's momentum list for both p' and q:
 *   spec_job, ins_job  indices into the job list;  op_begin, op_end, pairs,
 *   n_pairs, w as for c3pt_combine (host arrays, copied at creation);
 *   out  device complex128 [n_pairs][n_tau][op_end-op_begin][spin][64].
 *
 * c3pt_batch_create(jobs, n_jobs, combines, n_combines, k, n_mom, proj,
 *                   partial_budget, &batch)
 *   k[n_mom][3]     host momentum list shared by all jobs (1..128 momenta).
 *   proj            C3PT_PROJ_NATIVE (FP32), _SPLIT_F16 or _SPLIT_BF16.
 *   partial_budget  bytes of device memory for FP32 split-site partial sums;
 *                   jobs are grouped so that a group's partial sums fit
 *                   (0 = 16 GiB).  A job whose own partial sums exceed it is
 *                   rejected.
 *  Allocates device memory owned by the batch (queues, phase tables, partial
 *  sums, parameter tables); synchronizes the device work it enqueues.  On
 *  error nothing is kept and *batch is NULL.
 * c3pt_batch_run(batch, stream)    enqueue one replay on `stream`.  Every
 *  device buffer named at creation must stay allocated; its contents may change
 *  between runs.  Replays of one batch must not overlap (they share its
 *  queues and partial sums): use one stream, or synchronize.
 * c3pt_batch_info(batch, &n_items, &n_groups, &partial_bytes)   queue size,
 *  number of budget groups, partial-sum bytes held.
 * c3pt_batch_destroy(batch)   synchronizes the device and frees everything.
 */
#define C3PT_JOB_SPECTATOR_MESON   0
#define C3PT_JOB_SPECTATOR_BARYON  1
#define C3PT_JOB_INSERTION         2

typedef struct c3pt_job {
    int   kind;
    int   L[3];
    int   T;
    int   r[3];
    int   n_noise;
    const void* G;
    const void* G2;
    const void* eta;
    const void* const* G_t;
    const void* const* s_t;
    const void* const* U_t;
    const int*  taus;
    int   n_tau;
    int   n_ops;
    void* out;
} c3pt_job;

typedef struct c3pt_combine_job {
    int   spec_job;
    int   ins_job;
    int   op_begin;
    int   op_end;
    const double* w;
    const int*    pairs;
    int   n_pairs;
    void* out;
} c3pt_combine_job;

typedef struct c3pt_batch c3pt_batch;

int c3pt_batch_create(const c3pt_job* jobs, int n_jobs, const c3pt_combine_job* combines, int n_combines,
                      const int* k, int n_mom, int proj, unsigned long long partial_budget, c3pt_batch** batch);
int c3pt_batch_run(c3pt_batch* batch, void* stream);
int c3pt_batch_info(const c3pt_batch* batch, int* n_items, int* n_groups, unsigned long long* partial_bytes);
int c3pt_batch_destroy(c3pt_batch* batch);

/*
 * Serving: continuous batching of contraction requests.  A request is one
 * measurement of Eq. (8) on one lattice and source position: the spectator
 * part at t_f (meson, or the two nucleon spectators (u,u) and (u,d)), the
 * insertion part at every tau = t_src, t_src+1, ..., t_f (mod T), and the
 * combines (meson: S x I; nucleon, proton isovector: S(u,u) x I_d and
 * S(u,d) x I_u).  The propagators, noise and solutions stay resident in the
 * caller's device memory; requests only name them.
 *
 * c3pt_server_create(proj, arena, arena_bytes, step_bytes, max_active, stream, &server)
 *   proj        C3PT_PROJ_FACTORED, C3PT_PROJ_NATIVE (FP32), _SPLIT_F16 or
 *               _SPLIT_BF16 projection.
 *   arena       caller-owned device memory (256-byte aligned) from which the
 *               outputs of admitted requests are sub-allocated (first fit);
 *               it must outlive the server.
 *   step_bytes  device workspace for the FP32 partial sums of one step (>= 1 MiB);
 *               a request is cut into packets of at most step_bytes/4 (one
 *               noise vector of one timeslice must fit, else it is rejected).
 *   max_active  requests in flight at once.
 *   stream      hipStream_t every launch of the server goes to.
 * c3pt_server_submit(server, &req, &id)   validate and queue a request (host
 *   only; enqueues nothing).  Rejected with C3PT_EINVAL when its outputs (and,
 *   for the dense projections, its two phase tables) can never fit the arena,
 *   one noise vector of one timeslice exceeds a packet, or (factored) the
 *   momentum list does not factor.
 * c3pt_server_step(server, &n_active, &n_queued)   one iteration: admit
 *   queued requests while a slot and arena space are free, the one with the
 *   least work first (the one first in line is taken in turn once later ones
 *   have passed it 2 * max_active times); take packets from the active
 *   requests with the least remaining work first, each as many as fit, until
 *   the step workspace is full (a request that had no packet for four steps
 *   goes first); enqueue their contraction + projection (one launch per
 *   producer kind shared by all requests of the step), the FP64 reduction,
 *   and the combines of every request whose last packet ran, then an event
 *   marking it complete.  Returns after enqueueing; at most two steps are in
 *   flight (the call waits for the step before last).  The dense projections'
 *   phase tables live in the arena: built at the first admission that needs
 *   them, held while a request using them is active, then kept as a cache
 *   and evicted (least recently used first) when the arena needs the space.
 *   A request that cannot be admitted for a reason of its own (its tables
 *   cannot be built, or cannot fit even with nothing else active) leaves the
 *   queue as failed.
 * c3pt_server_set_step_work(server, max_work)   cap a step's work at max_work
 *   column blocks x sites (0, the default: no cap beyond the workspace).
 *   While no request waits for admission, a step ends where the next packet
 *   would pass the cap (it always takes one); with requests waiting, steps
 *   fill the workspace.  Requests admitted after the call are cut into
 *   packets of at most a quarter of the cap where one noise vector (of one
 *   timeslice) allows.  Shorter steps bound how long a new arrival waits for
 *   the steps in flight.  C3PT_EINVAL for a negative cap.
 * c3pt_server_poll(server, id)   1 when the request's results are complete on
 *   the device, 0 if not yet, or a negative status (a failed request: the
 *   status of its failure, with its message in c3pt_last_error).
 * c3pt_server_result(server, id, &res)   device pointers of the request's
 *   outputs inside the arena (valid once admitted; complete once polled 1):
 *     spec[p]  [n_noise][n_mom][192] meson, [n_noise][n_mom][3072] nucleon
 *     ins[p]   [n_noise][n_tau][n_ops][n_mom][192]
 *     comb[p]  [n_pairs][n_tau][n_ops][64 or 1024][64]
 *   p < n_parts (1 meson, 2 nucleon); layouts and orders as the single calls.
 * c3pt_server_release(server, id)   return the request's arena space (waits
 *   for its completion); also drops a request still queued or failed.
 * c3pt_server_info(server, &n_active, &n_queued, &largest_free_arena_bytes)
 * c3pt_server_destroy(server)   synchronizes the stream and frees the
 *   workspace; the arena (with the phase tables cached in it) stays the
 *   caller's.
 * A request's results do not depend on the other requests in flight: each
 * output element is summed over the same fixed site chunks in the same order.
 * One host thread drives a server.
 */
#define C3PT_REQ_MESON    0
#define C3PT_REQ_NUCLEON  1

typedef struct c3pt_request {
    int   kind;                 /* C3PT_REQ_MESON or C3PT_REQ_NUCLEON                        */
    int   L[3];
    int   T;
    int   r[3];                 /* spatial source position                                   */
    int   t_src;                /* first insertion timeslice                                 */
    int   t_f;                  /* sink timeslice (last insertion timeslice)                 */
    int   n_noise;
    int   n_ops;                /* 1 (local, 16 Gamma) or 5 (with the four D_nu)             */
    const void* const* G_t;     /* host [T] device slices: meson propagator, nucleon u       */
    const void* const* G2_t;    /* nucleon: host [T] device slices of the d propagator       */
    const void* const* s_t;     /* host [T] device [n_noise][12][V3] solutions               */
    const void* const* U_t;     /* host [T] device links when n_ops == 5, else NULL          */
    const void* eta;            /* device [n_noise][12][V3] noise on t_f                     */
    const int*  k;              /* host [n_mom][3] momenta (1..128), for p' and q            */
    int   n_mom;
    const int*  pairs;          /* host [n_pairs][2] (p', q) combine pairs, NULL = all       */
    int   n_pairs;
} c3pt_request;

typedef struct c3pt_result {
    void* spec[2];
    void* ins[2];
    void* comb[2];
    int   n_parts;
    int   n_tau;
    int   n_pairs;
} c3pt_result;

typedef struct c3pt_server c3pt_server;

int c3pt_server_create(int proj, void* arena, unsigned long long arena_bytes, unsigned long long step_bytes,
                       int max_active, void* stream, c3pt_server** server);
int c3pt_server_submit(c3pt_server* server, const c3pt_request* req, long long* id);
int c3pt_server_set_step_work(c3pt_server* server, double max_work);
int c3pt_server_step(c3pt_server* server, int* n_active, int* n_queued);
int c3pt_server_poll(c3pt_server* server, long long id);
int c3pt_server_result(c3pt_server* server, long long id, c3pt_result* res);
int c3pt_server_release(c3pt_server* server, long long id);
int c3pt_server_info(const c3pt_server* server, int* n_active, int* n_queued,
                     unsigned long long* largest_free_arena_bytes);
int c3pt_server_destroy(c3pt_server* server);

#ifdef __cplusplus
}
#endif

#endif /* C3PT_H */
