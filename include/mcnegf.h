/*
 * mcnegf.h -- C ABI of the MI355X (gfx950) library for the Monte Carlo NEGF method with
 * elastic Buttiker dephasing of Musland, Bergli and Flage-Larsen, "A Monte Carlo method
 * for solving the NEGF equations for electron transport".
 *
 * The library computes, for every energy E_k of a batch, in FP64 on the GPU:
 *   1. G^r = (E - H - Sigma_L - Sigma_R - Sigma_B)^{-1} of a W x L tight-binding wire by
 *      block-tridiagonal recursive Green's functions (Sec. III B; Sec. II A, Eq. (7));
 *   2. the walker's positive transition kernel: from probe j, weight gamma_i |G_ij|^2 to
 *      probe i and <psi_j|Gamma_r|psi_j> to lead r with psi_j = G|j> (step 6', Sec. II F,
 *      Eqs. (75), (76)); from a lead, the eigen-channel marginal of steps 3-4 (Eq. (39));
 *      one alias table per row;
 *   3. random walks that inject at a lead, hop between probe sites and are absorbed at a
 *      lead, counting exits; the estimator of the transmission is Tr Gamma_p A times
 *      [exit at q] (Sec. II E, Eq. (66));
 *   4. the effective L->R transmission either from the walk tallies (MC) or from the
 *      deterministic probe-conservation system (Sec. III C, Eq. (79)), and the current
 *      I = sum_k w_k T_eff(E_k) (midpoint quadrature, Sec. III C).
 * Further entry points, each declared below with its passage: the gradient of the DIRECT
 * current, batched walks over many built systems, energy-sampled walks, interpolated
 * step-6' rows, importance-sampled walks, the score-function gradient of the MC current,
 * inelastic walks (step 7') and one allocation-free walk.
 *
 * Model.  Sites i = x*W + y (x = 0..L-1 slices, y = 0..W-1), H_ii = V_i, H_ij = -t between
 * nearest neighbours, hard wall in y.  Leads attach to slices 0 (L) and L-1 (R).  Buttiker
 * probes: Sigma_B = diag(-(i/2) gamma_i) (Sec. III A, Eq. (77)).  Two lead models:
 *   0: clean semi-infinite leads with the wire's cross-section, hopping t, zero onsite,
 *      coupled by -t; surface Green's function taken at z = E + i*delta_lead*t;
 *   1: wide-band leads Sigma_p = -(i/2) Gamma_l on the end slice (Sec. III A, Eq. (78)).
 *
 * Conventions shared by every call.
 *   - Pointers named d_* are device pointers (HBM of the current HIP device); h_* are host.
 *     The caller owns every buffer.  The library allocates no device memory and keeps no
 *     global state; calls on different streams with different workspaces are independent.
 *   - All calls are asynchronous on `stream` except the host-only ones (the *_bytes size
 *     queries, mc_negf_interp_plan, mc_negf_plan_waves) and those that synchronise `stream`
 *     to return host results: mc_negf_current, mc_negf_current_interp,
 *     mc_negf_current_weighted, mc_negf_grad, mc_negf_status, mc_negf_batch_prepare,
 *     mc_negf_walk_batch_autotune (and mc_negf_profile_end, which waits for its events).
 *   - Every call returns an int32 status: 0 OK, > 0 warning, < 0 error (codes below).
 *     Arguments are validated on the host before any GPU work; on an error nothing is
 *     launched.  No C++ exception crosses the ABI.
 *   - Kernels record numerical trouble in a device status word inside the workspace; it is
 *     read by mc_negf_current / mc_negf_status.
 *   - Sizes: 1 <= W <= 32, 1 <= L, N = W*L, N + 2 <= 16320 (the alias build keeps 10 bytes
 *     per outcome of a row in one workgroup's LDS), 1 <= nE.
 */
#ifndef MCNEGF_H
#define MCNEGF_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------ */
#define MCNEGF_OK         0
#define MCNEGF_WTRUNC     1   /* some walks hit max_steps: the MC estimate is biased low  */
#define MCNEGF_WNUMERIC   2   /* a kernel invariant check (row sums) exceeded 1e-8 (1e-4   */
                              /* with MCNEGF_BUILD_FP32_PRODUCTS)                          */
#define MCNEGF_EINVAL    -1   /* bad size, null pointer, out-of-range parameter           */
#define MCNEGF_EWS       -2   /* workspace too small                                      */
#define MCNEGF_EHIP      -3   /* a HIP call failed; see mc_negf_last_hip_error()          */
#define MCNEGF_ENUMERIC  -4   /* NaN/Inf, singular RGF block or non-SPD probe system       */
#define MCNEGF_ENOTIMPL  -5   /* entry point not implemented                              */

/* ---- bits of the device status word ------------------------------------------------- */
#define MCNEGF_FLAG_NONFINITE  0x01u  /* NaN or Inf in G, the kernel or a solve           */
#define MCNEGF_FLAG_SINGULAR   0x02u  /* zero pivot while inverting an RGF block          */
#define MCNEGF_FLAG_ROWSUM     0x04u  /* a kernel row total differs from A_jj (or         */
                                      /* Tr Gamma_p A for a lead row) by more than 1e-8    */
                                      /* (1e-4 with MCNEGF_BUILD_FP32_PRODUCTS)            */
#define MCNEGF_FLAG_NOABSORB   0x08u  /* a lead has no open channel at some energy: its    */
                                      /* injection row is empty (its walkers exit at once  */
                                      /* into L and T = 0); happens outside the lead band, */
                                      /* where Tr Gamma_p <= 1e3 * delta_lead * t * W       */
#define MCNEGF_FLAG_TRUNC      0x10u  /* a walk reached max_steps                         */
#define MCNEGF_FLAG_NOTSPD     0x20u  /* non-positive pivot in the probe-system Cholesky  */
#define MCNEGF_FLAG_RANGE      0x40u  /* interpolated walks: an energy outside the built    */
                                      /* energies, or built energies that do not ascend    */

/* Number of per-energy lead scalars in mcnegf_kernel.lead, and their slots. */
#define MCNEGF_LEAD_NTERMS 8
#define MCNEGF_LEAD_TLL    0  /* Tr Gamma_L G_00 Gamma_L G_00^+                           */
#define MCNEGF_LEAD_TRL    1  /* Tr Gamma_R G_{L-1,0} Gamma_L G_{L-1,0}^+                 */
#define MCNEGF_LEAD_TLR    2  /* Tr Gamma_L G_{0,L-1} Gamma_R G_{0,L-1}^+                 */
#define MCNEGF_LEAD_TRR    3  /* Tr Gamma_R G_{L-1,L-1} Gamma_R G_{L-1,L-1}^+             */
#define MCNEGF_LEAD_CL     4  /* total weight of the L injection row (= Tr Gamma_L A)     */
#define MCNEGF_LEAD_CR     5  /* total weight of the R injection row (= Tr Gamma_R A)     */
#define MCNEGF_LEAD_TRGLA  6  /* Tr Gamma_L A from the diagonal block G_00                */
#define MCNEGF_LEAD_TRGRA  7  /* Tr Gamma_R A from G_{L-1,L-1}                            */

/* Tally slots of mc_negf_walk, per energy (int64, accumulated with +=). */
#define MCNEGF_TALLY_N         5
#define MCNEGF_TALLY_EXIT_L    0
#define MCNEGF_TALLY_EXIT_R    1
#define MCNEGF_TALLY_TRUNC     2
#define MCNEGF_TALLY_STEPS     3
#define MCNEGF_TALLY_STEPS2    4

/* Physical system (host struct, read during the call only). */
typedef struct mcnegf_system {
    int32_t W;            /* sites per slice, 1..32                                        */
    int32_t L;            /* number of slices, >= 1                                        */
    double  t;            /* hopping, > 0 (H_ij = -t)                                      */
    int32_t lead_model;   /* 0 clean semi-infinite leads, 1 wide-band leads                */
    double  gamma_l;      /* wide-band coupling Gamma_l (lead_model 1), >= 0               */
    double  delta_lead;   /* regulator in units of t: z = E + i*delta_lead*t (model 0), > 0 */
    uint32_t flags;       /* MCNEGF_BUILD_* bits; 0 builds everything                      */
} mcnegf_system;

/* mcnegf_system.flags.  MCNEGF_BUILD_NO_ALIAS: build G, the kernel rows' ingredients and
 * the lead terms but no alias tables (their workspace is not reserved; the handle's alias
 * and alias_lo are NULL).  Such a kernel serves the DIRECT current and its gradient;
 * mc_negf_walk and the MC mode of mc_negf_current reject it with MCNEGF_EINVAL. */
#define MCNEGF_BUILD_NO_ALIAS  0x1u
/* MCNEGF_BUILD_NO_DIRECT: reserve no workspace for the DIRECT solve (the handle's direct
 * and direct_vec are NULL); the DIRECT mode of mc_negf_current and mc_negf_grad reject such
 * a kernel with MCNEGF_EINVAL.  For Monte Carlo-only batches of large systems. */
#define MCNEGF_BUILD_NO_DIRECT 0x2u
/* MCNEGF_BUILD_FP32_PRODUCTS: the block products of the full inverse (the sweeps that
 * produce every block of G from the RGF blocks, Sec. III B) run as FP32 complex products on
 * the matrix cores, with the column state in FP32; the RGF blocks, |G_ij|^2, the exit
 * weights, the lead terms, the alias tables, the probe solve and all tallies stay FP64.
 * Only W = 16 and W = 32 (mc_negf_build_kernel returns MCNEGF_EINVAL for other widths);
 * |G_ij|^2 then carries FP32 rounding (relative error of order 1e-6 after hundreds of
 * slices), and so do the currents, and the probe solve inside mc_negf_grad on such a build
 * (its complex G is recomputed in FP64); MCNEGF_BUILD_FP32_REFINE adds one refinement step. */
#define MCNEGF_BUILD_FP32_PRODUCTS 0x4u
/* MCNEGF_BUILD_FP32_REFINE (with MCNEGF_BUILD_FP32_PRODUCTS only): the FP32 sweeps store every
 * block of G0, and one step of iterative refinement of (E - H - Sigma) G = I (Sec. II A,
 * Eq. (7)) corrects it before |G|^2, the exit weights and the corners are formed: the residual
 * I - A G0 in FP64 (5-point stencil and lead blocks), the correction solved in FP32 with the
 * block LU of the left-connected RGF blocks, G1 = G0 + correction in FP64.  |G_ij|^2 and the
 * currents then agree with an FP64 build to about 1e-12 relative.  The refinement also
 * rewrites the diagonal blocks and A_jj from G1.  The workspace grows by 24 bytes per entry of
 * G for 8 energies at a time (refined 8 energies per pass). */
#define MCNEGF_BUILD_FP32_REFINE 0x8u
/* MCNEGF_BUILD_FP32_SWEEPS (with MCNEGF_BUILD_FP32_PRODUCTS only): the left and right RGF
 * sweeps (g_k = (A_k - t^2 g_{k-1})^{-1}, Sec. III B) also run in FP32; the diagonal blocks
 * are then formed in FP64 from the FP32 sweep blocks.  Errors grow with the length: at
 * W = 32, L = 500 about 2e-5 relative in T_eff without refinement and 5e-11 with
 * MCNEGF_BUILD_FP32_REFINE (whose correction solve then uses the FP32 blocks). */
#define MCNEGF_BUILD_FP32_SWEEPS 0x10u

/*
 * Handle filled by mc_negf_build_kernel: shapes plus device pointers into the caller's
 * workspace (valid while the workspace lives and until the next build into it).  All
 * device arrays are FP64 unless stated.  Row-major; energy index outermost.
 */
typedef struct mcnegf_kernel {
    int32_t  W, L, N, n_out, nE;  /* n_out = N + 2: probes 0..N-1, lead L = N, lead R = N+1 */
    int32_t  lead_model;
    double   t;
    double   delta_lead;    /* copied from the system                                       */
    int64_t  alias_pitch;   /* entries per alias row (>= n_out, multiple of 16)            */
    int64_t  p_pitch;       /* doubles per row of P (>= N, multiple of 16)                 */
    const double* energies; /* [nE], borrowed from the caller                              */
    const double* gamma;    /* [N], borrowed from the caller                               */
    uint32_t* alias;        /* [nE][n_out][alias_pitch] packed alias entries:              */
                            /*  bits 31..16 = thr >> 16, bits 15..0 = alias                 */
    uint16_t* alias_lo;     /* [nE][n_out][alias_pitch] thr & 0xFFFF.  Bucket c keeps       */
                            /*  outcome c when a uniform 32-bit word r satisfies r < thr,   */
                            /*  else goes to outcome alias (the low part of thr is read     */
                            /*  only when r >> 16 == thr >> 16)                             */
    double*   P;            /* [nE][N][p_pitch]  |G_ij|^2                                  */
    double*   wL;           /* [nE][N]  <psi_j|Gamma_L|psi_j>, psi_j = G|j>                 */
    double*   wR;           /* [nE][N]  <psi_j|Gamma_R|psi_j>                               */
    double*   Adiag;        /* [nE][N]  A_jj = -2 Im G_jj                                  */
    double*   lead;         /* [nE][MCNEGF_LEAD_NTERMS]                                    */
    double*   sigma;        /* [nE][W][W] complex (re, im) lead self-energy (both leads)   */
    double*   gam_lead;     /* [nE][W][W] Gamma = i(Sigma - Sigma^+), real symmetric       */
    double*   gL;           /* [nE][L][W][W] complex: left-connected blocks                */
    double*   gR;           /* [nE][L][W][W] complex: right-connected blocks               */
    double*   Gd;           /* [nE][L][W][W] complex: diagonal blocks G_kk                  */
    double*   corner;       /* [nE][2][W][W] complex: G_{L-1,0} and G_{0,L-1}              */
    double*   direct;       /* [nE][p_pitch+2][p_pitch] Cholesky factor of the bordered     */
                            /* scaled probe system (DIRECT mode), lower part                */
    double*   direct_vec;   /* [nE][4][N] scratch vectors (DIRECT mode)                    */
    double*   reduce;       /* [nE + 8] scratch for current reductions                     */
    uint32_t* status;       /* device status word (MCNEGF_FLAG_* bits)                     */
    uint32_t* counters;     /* [64] walker work counters                                   */
    void*     ws;           /* workspace base                                              */
    uint64_t  ws_bytes;
} mcnegf_kernel;

/*
 * Bytes of device workspace that mc_negf_build_kernel needs for `sys` and nE energies.
 * Host only; no GPU work.  Returns MCNEGF_EINVAL for invalid sizes or null pointers.
 */
int32_t mc_negf_workspace_bytes(const mcnegf_system* sys, int32_t nE, uint64_t* bytes_out);

/*
 * Build the per-energy Green's functions, transition kernels and alias tables (no alias
 * tables when sys->flags has MCNEGF_BUILD_NO_ALIAS).
 *   sys        physical system (host).
 *   d_onsite   [N] device, V_i, slice-major.
 *   d_gamma    [N] device, gamma_i >= 0 (dephasing rate of the probe on site i); the
 *              kernel handle keeps this pointer, so it must stay valid while k is used.
 *   d_energies [nE] device, energies E_k (units of t); kept by the handle as well.
 *   d_ws       device workspace of ws_bytes >= mc_negf_workspace_bytes(sys, nE), 256-byte
 *              aligned; owned by the caller; overwritten.
 *   out        host handle, filled on success.
 * Stages (all on `stream`): lead self-energies Sigma_p, Gamma_p = i(Sigma_p - Sigma_p^+)
 * (Sec. II A, Eqs. (9)-(11); wide band: Sec. III A, Eq. (78)); left/right RGF sweeps and the
 * diagonal blocks of G^r = (E - H - Sigma)^{-1} (Sec. III B; Eq. (7)); the off-diagonal
 * blocks streamed into |G_ij|^2, <psi_j|Gamma_r|psi_j> and the corner blocks (the step-6'
 * weights, Sec. II F, Eqs. (75), (76)); lead transmissions and the injection rows (steps 3-4,
 * Eq. (39)); one alias table per kernel row.  Asynchronous.
 */
int32_t mc_negf_build_kernel(const mcnegf_system* sys, const double* d_onsite,
                             const double* d_gamma, const double* d_energies, int32_t nE,
                             void* d_ws, uint64_t ws_bytes, mcnegf_kernel* out,
                             hipStream_t stream);

/*
 * Random walks on the alias tables of k (Sec. II F, step 6' repeated until a lead is drawn).
 *   seed, realization  key of the Philox4x32-10 streams; realization < 2^30.
 *   inject_lead        0: walkers start in the L injection row, 1: in the R row.
 *   walker_begin, n_walkers_per_energy  walker indices [walker_begin, walker_begin + n)
 *                      are walked at every energy; walker_begin + n < 2^32 (the range
 *                      end is held in 32 bits), else MCNEGF_EINVAL.
 *   max_steps          walks still inside after max_steps draws are counted as truncated
 *                      (the injection draw counts as one step); >= 1.
 *   d_tallies          [nE][MCNEGF_TALLY_N] int64 device, accumulated (+=).
 * Stream layout: key = (seed low, seed high); block j of walker w at energy index e has
 * counter (j, w, e, (realization << 1) | inject_lead); step n uses words 2(n&1), 2(n&1)+1 of
 * block n>>1 as (a, b); bucket c = (a * n_out) >> 32 with Lemire's rejection (the r-th redraw
 * of step n takes word 0 of the block with counter (n, w, e, tag | 2^31) and key
 * (key0, key1 ^ r)); outcome = b < thr[c] ? c : alias[c].  Results are a pure function of
 * (tables, seed, realization, inject_lead, walker range); tallies of [a, b) plus [b, c)
 * equal those of [a, c) exactly.  Asynchronous.
 */
int32_t mc_negf_walk(const mcnegf_kernel* k, uint64_t seed, uint32_t realization,
                     uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers_per_energy,
                     uint32_t max_steps, int64_t* d_tallies, hipStream_t stream);

/*
 * Effective transmission per energy and the current (Sec. II E, Eq. (66); Sec. III C).
 *   mode 0 (MC): from d_tallies of walks injected at `inject_lead`:
 *     p_k = exits at the other lead / walkers,  T_k = c_p p_k,
 *     sigma_k = c_p sqrt(p_k (1 - p_k) / (walkers - 1)),  c_p = row total of injection row p.
 *   mode 1 (DIRECT): solve (diag(gamma_j A_jj) - T_PP) f = T_Pp by Cholesky on the GPU and
 *     T_k = T_qp + sum_j T_qj f_j; sigma_k = 0.  d_tallies is ignored (may be null).
 *   mode 2 (energy-sampled MC, tallies of mc_negf_walk_sampled with the same weights): the
 *     constant estimator X = W c_p(E_k) [exit at q] over all N walkers, W = sum_k w_k:
 *     I = (W / N) sum_k c_p,k R_k (R_k exits at q at energy k), sigma_I^2 = (W^2 S2 / N - I^2)
 *     / (N - 1) with S2 = sum_k c_p,k^2 R_k; T_k and sigma_k per energy as in mode 0.
 *   d_weights [nE] device quadrature weights w_k; d_T, d_sigmaT [nE] device outputs.
 *   h_I_sigma [2] host output: I = sum_k w_k T_k and sqrt(sum_k w_k^2 sigma_k^2) (modes 0, 1),
 *     or the mode-2 I and sigma_I.
 * Synchronises `stream`, then reads the device status word: returns MCNEGF_ENUMERIC if a
 * NONFINITE, SINGULAR or NOTSPD bit is set, MCNEGF_WTRUNC if TRUNC is set (MC modes),
 * MCNEGF_WNUMERIC if ROWSUM is set, else MCNEGF_OK.
 */
int32_t mc_negf_current(const mcnegf_kernel* k, int32_t mode, uint32_t inject_lead,
                        const int64_t* d_tallies, const double* d_weights, double* d_T,
                        double* d_sigmaT, double* h_I_sigma, hipStream_t stream);

/*
 * Bytes of device workspace mc_negf_grad needs for the built kernel `k` (host only): the
 * complex G [chunk][N][p_pitch], the adjoint solves [chunk][N][roundup(N + W, 16)] and
 * O(chunk N) vectors for `chunk` energies at a time, plus O(nE N) per-energy derivatives.
 * mc_negf_grad_workspace_bytes gives the size for all energies at once (chunk = nE),
 * mc_negf_grad_workspace_bytes_chunk for 1 <= chunk <= nE.  MCNEGF_EINVAL for a bad handle.
 */
int32_t mc_negf_grad_workspace_bytes(const mcnegf_kernel* k, uint64_t* bytes_out);
int32_t mc_negf_grad_workspace_bytes_chunk(const mcnegf_kernel* k, int32_t chunk,
                                           uint64_t* bytes_out);

/*
 * Gradient of the DIRECT current I = sum_k w_k T_eff(E_k) (Sec. III C, Eq. (79) read as the
 * diagonal of Eq. (8)) with respect to the onsite potentials V_i (H_ii) and the dephasing
 * rates gamma_i (Sigma_s,ii = -(i/2) gamma_i, Sec. III A, Eq. (77)), by the adjoint of the
 * probe system and of G = (E - H - Sigma)^{-1} (dI/deta for uniform gamma_i = eta is the sum
 * of dI/dgamma_i).  The lead self-energies are held fixed.
 *   k            handle from mc_negf_build_kernel (reads its tables; reruns the DIRECT solve).
 *   inject_lead  0: T_RL (f_L = 1), 1: T_LR.
 *   d_weights    [nE] device, quadrature weights w_k.
 *   d_gws        device workspace, caller-owned: with mc_negf_grad_workspace_bytes bytes all
 *                energies are differentiated at once; a smaller one (at least the one-energy
 *                size of mc_negf_grad_workspace_bytes_chunk) takes the energies in the largest
 *                chunks it holds, regenerating each chunk's G from the stored RGF blocks.
 *   d_dI_dV      [N] device output dI/dV_i;  d_dI_dgamma [N] device output dI/dgamma_i.
 *   h_I          host output, the DIRECT current I.
 * Needs a kernel built with the DIRECT workspace (else MCNEGF_EINVAL); any W <= 32 and N.
 * Synchronises `stream`; status as mc_negf_current in DIRECT mode.  MCNEGF_EWS if the
 * workspace is too small; MCNEGF_EHIP if a launch fails.
 */
int32_t mc_negf_grad(const mcnegf_kernel* k, uint32_t inject_lead, const double* d_weights,
                     void* d_gws, uint64_t gws_bytes, double* d_dI_dV, double* d_dI_dgamma,
                     double* h_I, hipStream_t stream);

/*
 * Score-function gradient of the Monte Carlo current: the derivative of the reweighted path
 * estimator of Eq. (66) (Sec. V A, "Improved estimator": walks drawn at the current
 * parameters, weighted by their likelihood ratio at perturbed ones).  For walks injected at p,
 *   dT/dtheta ~ (c_p / N_w) d/dtheta [ sum_so C_so K_so / K_so(0) - sum_s n_s A_ss / A_ss(0) ]
 * with C_so the steps s -> o of the walks that reached q, n_s = sum_o C_so, K the kernel
 * weights (Eqs. (75), (76)), theta = V_i or gamma_i; its mean is the exact derivative of the
 * current (the library's mc_negf_grad gives that exactly).
 * mc_negf_walk_counts_bytes (host only): bytes of the counts array, nE * n_out^2 * 4.
 * mc_negf_walk_counts: walkers [walker_begin, walker_begin + n_walkers) (< 2^32) at every
 *   energy, drawing exactly as mc_negf_walk; adds to d_counts [nE][n_out][n_out] (uint32,
 *   device, outcome-major: d_counts[e][o][s] counts steps s -> o; caller-owned, zeroed by the
 *   caller before the first call) the steps of every walk that exits at q, and their exit
 *   counts to d_tallies as mc_negf_walk.  Each entry is a 32-bit count (it wraps beyond
 *   2^32 - 1 steps s -> o; split larger runs and sum the gradients).  Needs a kernel with
 *   alias tables.  Asynchronous.
 * mc_negf_grad_mc: from those counts and tallies, d_dI_dV [N] and d_dI_dgamma [N] (device)
 *   = sum_k w_k times the estimate above at energy k (dgamma: gamma_i > 0; for gamma_i = 0 the
 *   walks never enter site i and the explicit term is taken as 0).  d_gws: the workspace of
 *   mc_negf_grad (mc_negf_grad_workspace_bytes[_chunk]; energies in chunks as there).  Any
 *   W <= 32; the kernel needs no DIRECT workspace.  Asynchronous; MCNEGF_EINVAL for bad
 *   arguments, MCNEGF_EWS for a workspace below the one-energy size, MCNEGF_EHIP on a failed
 *   launch.
 */
int32_t mc_negf_walk_counts_bytes(const mcnegf_kernel* k, uint64_t* bytes_out);
int32_t mc_negf_walk_counts(const mcnegf_kernel* k, uint64_t seed, uint32_t realization,
                            uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers,
                            uint32_t max_steps, uint32_t* d_counts, int64_t* d_tallies,
                            hipStream_t stream);
int32_t mc_negf_grad_mc(const mcnegf_kernel* k, uint32_t inject_lead, const uint32_t* d_counts,
                        const int64_t* d_tallies, const double* d_weights, void* d_gws,
                        uint64_t gws_bytes, double* d_dI_dV, double* d_dI_dgamma,
                        hipStream_t stream);

/*
 * Inelastic walks: step 7' of Sec. II F.  With Buttiker's approximation and an energy-changing
 * coupling lambda~_i(E, E'), a walker that step 6' sends to probe i at energy E_n draws its next
 * energy from p(E) = lambda~_i(E, E_n) A_ii(E) / (integral over E of the same) (Eq. (74),
 * the probability that follows the choice of the index, Sec. II F) and continues from probe
 * i's row at that energy.  The coupling here is a set of lines on the energy grid of the handle,
 *   lambda~_i(E, E_n) = sum_k lambda_k delta(E - E_n - Delta_k),  Delta_k = offsets[k] grid steps,
 * the same for every site (e.g. an elastic line at 0 and phonon emission / absorption lines at
 * -m / +m); a line that leaves the grid has weight 0.  The energies must be evenly spaced for
 * a line to be a fixed energy transfer (not checked).  The dephasing rates gamma_i of the build
 * stay the caller's: condition (iv) of Sec. II F (Eq. (69)) ties them to the coupling, but the
 * walk is a proper Markov chain either way (step 7' is normalised by its own sum).
 *   n_lines    1 .. 8 lines; h_offsets [n_lines] host, |offset| < nE; h_lambda [n_lines] host,
 *              finite, >= 0, and from every energy some line of positive weight stays on the grid
 *              (else MCNEGF_EINVAL).
 * mc_negf_energy_table_bytes (host only): nE * N * n_lines * 8.
 * mc_negf_energy_table: d_table [nE][N][n_lines] (uint64, device, caller-owned) from the
 *   handle's A_jj: x_k = lambda_k A_ii(E_e + Delta_k) summed in order (FP64, cum_k), then
 *   t_k = floor(2^32 cum_k / cum_last).  A non-positive or non-finite total writes 2^32
 *   everywhere (line 0 is drawn) and sets MCNEGF_FLAG_NONFINITE.  MCNEGF_EWS if table_bytes is
 *   too small.  Asynchronous.
 * mc_negf_walk_inelastic: walkers [walker_begin, walker_begin + n_walkers) (< 2^32) injected at
 *   lead inject_lead at every energy e0 of the handle (nE <= 4096, one energy's alias table
 *   below 2^32 entries), on its alias tables, with
 *   step 7' drawn from d_table (the offsets must be those the table was built with): the first
 *   k with r < t_k (k = n_lines - 1 if none) for the 32-bit word r of the step.  A walker keeps
 *   the random stream of its injection energy: step-6' words and Lemire redraws as
 *   mc_negf_walk at e0; the word of step n's energy draw is word (n & 3) of Philox4x32-10 at
 *   counter (n >> 2, w, e0, tag), key (~key0, key1).  With the single line Delta = 0 the walks
 *   are mc_negf_walk's.  Adds to d_tallies [nE][MCNEGF_TALLY_N] (device, per injection energy,
 *   as mc_negf_walk; mc_negf_current in mode 0 gives the current: a walker scores c_p(e0) at an
 *   exit at q) and to d_hist [2][nE][nE] (int64, device, caller-zeroed): hist[r][e0][e] counts
 *   walkers from e0 absorbed at lead r with energy e.  A table that sends a walk off the grid
 *   ends it as truncated and sets MCNEGF_FLAG_RANGE; max_steps truncation sets
 *   MCNEGF_FLAG_TRUNC.  table_bytes: the size of d_table (MCNEGF_EWS below
 *   mc_negf_energy_table_bytes).  Asynchronous.
 * mc_negf_spectrum: d_spectrum [2][nE] (device) = the energy-resolved current
 *   S[r][e] = sum_e0 w_e0 c_p(e0) hist[r][e0][e] / N_e0 (N_e0 the walkers injected at e0);
 *   sum_e S[q][e] is the current of the tallies.  Asynchronous.
 * All three launch one kernel each and are capturable in a HIP graph (mc_negf_graph_begin).
 */
int32_t mc_negf_energy_table_bytes(const mcnegf_kernel* k, int32_t n_lines, uint64_t* bytes_out);
int32_t mc_negf_energy_table(const mcnegf_kernel* k, int32_t n_lines, const int32_t* h_offsets,
                             const double* h_lambda, uint64_t* d_table, uint64_t table_bytes,
                             hipStream_t stream);
int32_t mc_negf_walk_inelastic(const mcnegf_kernel* k, int32_t n_lines, const int32_t* h_offsets,
                               const uint64_t* d_table, uint64_t table_bytes, uint64_t seed,
                               uint32_t realization,
                               uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers,
                               uint32_t max_steps, int64_t* d_tallies, int64_t* d_hist,
                               hipStream_t stream);
int32_t mc_negf_spectrum(const mcnegf_kernel* k, uint32_t inject_lead, const int64_t* d_tallies,
                         const int64_t* d_hist, const double* d_weights, double* d_spectrum,
                         hipStream_t stream);

/*
 * Energy-sampled walks (Sec. II F step 2: the starting energy drawn from a density h; with
 * h proportional to the quadrature weights the estimator of Eq. (66) becomes the constant
 * W c_p(E_0) [exit at q], W = sum_k w_k — the paper's choice h = Th(E) when w_k = Th(E_k) dE).
 * Walker w of [walker_begin, walker_begin + n_walkers) draws its energy index k with
 * probability d_weights[k] / W from Philox4x32-10 counter (0, w, 0xFFFFFFFF, tag) (words 0-1
 * as a 53-bit uniform u; k = the first index with cdf_{k+1} > u cdf_nE, cdf the running sum
 * of the weights in index order) and then walks exactly as in mc_negf_walk at energy k; its
 * counts go to d_tallies[k] (accumulated).  The walkers are sorted by energy on the device
 * and walked in one launch; everything is asynchronous (capturable).  Estimate the current
 * with mc_negf_current mode 2.  Needs nE <= 16384, walker_begin + n_walkers < 2^32 and a
 * kernel with alias tables; d_scratch (caller-owned, 256-byte aligned) of
 * >= mc_negf_walk_sampled_bytes(k, n_walkers) bytes.
 * A negative or non-finite weight counts as 0 and sets MCNEGF_FLAG_NONFINITE.
 */
int32_t mc_negf_walk_sampled_bytes(const mcnegf_kernel* k, uint64_t n_walkers,
                                   uint64_t* bytes_out);
int32_t mc_negf_walk_sampled(const mcnegf_kernel* k, uint64_t seed, uint32_t realization,
                             uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers,
                             uint32_t max_steps, const double* d_weights, int64_t* d_tallies,
                             void* d_scratch, uint64_t scratch_bytes, hipStream_t stream);

/*
 * mc_negf_walk_sampled without a scratch argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments (less d_scratch, scratch_bytes), same walks and the same
 * tallies bit for bit as mc_negf_walk_sampled; no device memory is allocated or freed.  Its
 * scratch is one fixed array of MCNEGF_STATIC_SCRATCH_BYTES per device, held from the first
 * call on that device until the process ends; returns MCNEGF_EWS when
 * mc_negf_walk_sampled_bytes(k, n_walkers) exceeds it (e.g. 256 energies: up to about 8e6
 * walkers per call).  Every call on a device shares that device's array, so calls that
 * overlap on one device (concurrent streams or threads) race; calls in order on one stream
 * do not.  Nothing in the array needs to start at zero.  Asynchronous.
 */
#define MCNEGF_STATIC_SCRATCH_BYTES (64ull << 20)
int32_t mc_negf_walk_sampled_noalloc(const mcnegf_kernel* k, uint64_t seed,
                                     uint32_t realization, uint32_t inject_lead,
                                     uint64_t walker_begin, uint64_t n_walkers,
                                     uint32_t max_steps, const double* d_weights,
                                     int64_t* d_tallies, hipStream_t stream);

/*
 * Interpolated step-6' probabilities across energies (Sec. V A, "Interpolation").  Walks at
 * energies between the built ones take the rows of their two neighbouring built energies
 * E_lo <= E < E_hi mixed linearly: (1 - alpha) p(E_lo) + alpha p(E_hi), alpha = (E - E_lo) /
 * (E_hi - E_lo) stored as the 32-bit threshold min(floor(alpha 2^32), 2^32 - 1) (at the last
 * built energy alpha = 0).  The built energies (the kernel's d_energies) must ascend.  An
 * interval is fit for interpolation when its two energies' normalised rows are close; energies
 * in the other intervals are to be built exactly (they become built energies themselves).
 *
 * mc_negf_interp_distances: d_dist[e] (device, [nE - 1]) = the largest, over the kernel rows
 *   (probes and both injection rows), L1 distance sum_i |p_i(E_e) - p_i(E_e+1)| of the
 *   normalised rows (2 for a row without weight).  Needs nE >= 2; works on a kernel built with
 *   or without alias tables.  Asynchronous.
 * mc_negf_interp_plan (host only): the fine energies h_fine[f] that must be built exactly: those
 *   strictly inside an interval [h_nodes[e], h_nodes[e + 1]) with h_dist[e] > tol (or NaN).
 *   Writes their indices (ascending) to h_exact[0 .. *n_exact - 1] (room for nF).  MCNEGF_EINVAL
 *   for nodes that do not ascend or a fine energy outside [h_nodes[0], h_nodes[nN - 1]].
 * mc_negf_walk_interp: walkers [walker_begin, walker_begin + n) (< 2^32) at each of the nF fine
 *   energies d_fine_energies (device) on the kernel's alias tables, drawing each step from the
 *   mixture: one Philox4x32-10 block of counter (n, w, f | 2^31, tag) per step n of walker w at
 *   fine energy f, words 0 and 1 as in mc_negf_walk, word 2 < threshold(alpha_f) takes E_hi's
 *   table (Lemire redraws: counter (n, w, f | 2^31, tag | 2^31), key (key0, key1 ^ r)).
 *   d_tallies [nF][MCNEGF_TALLY_N] (accumulated).  Asynchronous; a fine energy outside the built
 *   ones sets MCNEGF_FLAG_RANGE (it is walked at the nearest end).
 * mc_negf_current_interp: T_f = c_f p_f and sigma_f as in mc_negf_current mode 0 with the
 *   interpolated row total c_f = (1 - alpha_f) c_p(E_lo) + alpha_f c_p(E_hi), and
 *   I = sum_f w_f T_f, sigma_I (h_I_sigma).  d_weights, d_T, d_sigmaT: [nF] device.  Synchronises
 *   the stream; MCNEGF_EINVAL if MCNEGF_FLAG_RANGE is set, else as mc_negf_current mode 0.
 */
int32_t mc_negf_interp_distances(const mcnegf_kernel* k, double* d_dist, hipStream_t stream);
int32_t mc_negf_interp_plan(const double* h_nodes, int32_t nN, const double* h_dist,
                            const double* h_fine, int32_t nF, double tol, int32_t* h_exact,
                            int32_t* n_exact);
int32_t mc_negf_walk_interp(const mcnegf_kernel* k, const double* d_fine_energies, int32_t nF,
                            uint64_t seed, uint32_t realization, uint32_t inject_lead,
                            uint64_t walker_begin, uint64_t n_walkers_per_energy,
                            uint32_t max_steps, int64_t* d_tallies, hipStream_t stream);
int32_t mc_negf_current_interp(const mcnegf_kernel* k, const double* d_fine_energies,
                               int32_t nF, uint32_t inject_lead, const int64_t* d_tallies,
                               const double* d_weights, double* d_T, double* d_sigmaT,
                               double* h_I_sigma, hipStream_t stream);

/*
 * Importance-sampled walks (Sec. V A, "Improved estimator": step-6' probabilities p replaced
 * by other probabilities p', the estimator of Eq. (66) weighted by p / p' along the path).
 * For a bias b over the n_out outcomes of each energy,
 *   p'_ij = p_ij b_j / rho_i,   rho_i = sum_j p_ij b_j,
 * so a step i -> j multiplies the path's likelihood ratio by rho_i / b_j.  A walk injected at
 * lead p that exits at the other lead q scores c_p times the product of its ratios, any other
 * walk scores 0.  The mean is T_qp whenever b is finite and non-negative, positive at q and at
 * every probe a walk to q can pass through; b = P(exit at q | state) gives zero variance, and
 * b = 1 is the plain walk.  A poor b can make the variance infinite (the sample variance then
 * understates the error).
 *
 * mc_negf_weighted_tables_bytes (host only): device bytes of the modified tables of kernel k.
 * mc_negf_weighted_tables: from the kernel k (built with or without its own alias tables,
 *   MCNEGF_BUILD_NO_ALIAS) and d_bias [nE][n_out] (device, FP64), writes into d_tables
 *   (caller-owned device memory of >= that size, 256-byte aligned) the alias tables of the
 *   modified rows in the kernel's format - packed entries [nE][n_out][alias_pitch] (uint32),
 *   then the low threshold bits (uint16, same shape), then rho [nE][n_out] (FP64), each part
 *   starting at a multiple of 256 bytes - and the injection rows' totals c_p into the lead
 *   terms (MCNEGF_LEAD_CL, _CR, the values the kernel's own build stores).  A negative or
 *   non-finite bias entry sets MCNEGF_FLAG_NONFINITE.  Asynchronous.
 * mc_negf_walk_weighted_bytes (host only): device scratch bytes mc_negf_walk_weighted needs for
 *   n_walkers walkers per energy (16 bytes per energy per 2048 walkers).
 * mc_negf_walk_weighted: walkers [walker_begin, walker_begin + n_walkers) (< 2^32) at every
 *   energy, drawing exactly as mc_negf_walk does, on the modified tables d_tables (as written
 *   above, tables_bytes their size) with the same d_bias; adds their exit counts to d_tallies
 *   [nE][MCNEGF_TALLY_N] (int64, as mc_negf_walk) and to d_wsum [nE][2] (FP64) the sum of the
 *   scores / c_p and the sum of their squares.  The sums for a given walker range do not
 *   depend on scheduling.  d_scratch: caller-owned, 256-byte aligned, >=
 *   mc_negf_walk_weighted_bytes.  Asynchronous.
 * mc_negf_current_weighted: per energy, with N_k walkers and score sums S1, S2 (without c_p),
 *   T_k = c_p S1 / N_k and sigma_k = c_p sqrt(s^2 / N_k), s^2 = (S2 - S1^2 / N_k) / (N_k - 1);
 *   I and sigma_I as mc_negf_current.  Synchronises `stream`; status as mc_negf_current in
 *   MC mode.
 * All four: MCNEGF_EINVAL for a bad handle or argument, MCNEGF_EWS for a short or misaligned
 * buffer, MCNEGF_EHIP if a launch fails.
 */
int32_t mc_negf_weighted_tables_bytes(const mcnegf_kernel* k, uint64_t* bytes_out);
int32_t mc_negf_weighted_tables(const mcnegf_kernel* k, const double* d_bias, void* d_tables,
                                uint64_t tables_bytes, hipStream_t stream);
int32_t mc_negf_walk_weighted_bytes(const mcnegf_kernel* k, uint64_t n_walkers,
                                    uint64_t* bytes_out);
int32_t mc_negf_walk_weighted(const mcnegf_kernel* k, const void* d_tables, uint64_t tables_bytes,
                              const double* d_bias, uint64_t seed, uint32_t realization,
                              uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers,
                              uint32_t max_steps, int64_t* d_tallies, double* d_wsum,
                              void* d_scratch, uint64_t scratch_bytes, hipStream_t stream);
int32_t mc_negf_current_weighted(const mcnegf_kernel* k, uint32_t inject_lead,
                                 const int64_t* d_tallies, const double* d_wsum,
                                 const double* d_weights, double* d_T, double* d_sigmaT,
                                 double* h_I_sigma, hipStream_t stream);

/*
 * Like mc_negf_current, but asynchronous and capturable in a HIP graph: I and the standard
 * error go to d_I_sigma ([2] device) instead of the host, nothing is synchronised and the
 * status word is left for mc_negf_status to read.  Same argument rules and errors
 * (MCNEGF_EINVAL, MCNEGF_EHIP) as mc_negf_current.
 */
int32_t mc_negf_current_async(const mcnegf_kernel* k, int32_t mode, uint32_t inject_lead,
                              const int64_t* d_tallies, const double* d_weights, double* d_T,
                              double* d_sigmaT, double* d_I_sigma, hipStream_t stream);

/*
 * Batched walks over many built kernels (systems of different sizes; every energy of every
 * kernel is one unit), in one persistent launch (Sec. II F step 6', walked as in
 * mc_negf_walk).  The tallies equal those of mc_negf_walk on each kernel with the same seed,
 * realization, injection lead and walker range, bit for bit, for every launch shape.
 *
 * mc_negf_batch_bytes: device bytes of the batch buffer for these kernels (host only).
 * mc_negf_batch_prepare: write the unit table for `kernels` (each built with alias tables)
 *   into d_buf (caller-owned device memory of >= mc_negf_batch_bytes, 256-byte aligned) and
 *   fill *out.  realizations[i] and inject_lead form kernel i's Philox tag as in
 *   mc_negf_walk; d_tallies[i] is kernel i's [nE][MCNEGF_TALLY_N] tally array (device,
 *   accumulated).  Copies the table from the host and synchronises `stream`: call it before
 *   a graph capture, not inside one.  The kernels' workspaces must outlive the batch.
 * mc_negf_walk_batch: walk walkers [walker_begin, walker_begin + n_walkers_per_energy)
 *   (walker_begin + n_walkers_per_energy < 2^32) of
 *   every unit; one kernel launch, asynchronous, capturable.  cfg NULL = the default shape.
 * mc_negf_walk_batch_autotune: time every candidate launch shape (walker slots per lane
 *   1-4, workgroup size 64 / 256, chunk of 2 / 8 / 32 walks per slot, XCD groups 1 / 8) on
 *   this batch with n_walkers_per_energy walkers, counting into the batch buffer's scratch
 *   tallies (the kernels' tallies are untouched), and return the fastest in *best and its
 *   time in *best_ms.  Synchronises `stream`.
 * Errors: MCNEGF_EINVAL (null pointers, a kernel without alias tables, a bad shape),
 * MCNEGF_EWS (buffer too small or misaligned), MCNEGF_EHIP.
 */
typedef struct mcnegf_walk_config {
    int32_t slots;           /* walker slots per lane, 1..4                                 */
    int32_t wg_size;         /* threads per workgroup: 64, 128, 256 or 512                  */
    int32_t groups;          /* 1, or 8 (units spread over the XCDs, unit u on XCD u % 8)  */
    int32_t walks_per_slot;  /* chunk = 64 * slots * walks_per_slot walkers (chunk == 0)    */
    int32_t chunk;           /* walkers per chunk; 0 = from walks_per_slot                  */
} mcnegf_walk_config;

typedef struct mcnegf_batch {
    void*    d_units;           /* device unit table (inside the batch buffer)             */
    int64_t* d_scratch_tallies; /* [n_units][MCNEGF_TALLY_N] (inside the batch buffer)     */
    uint32_t n_units;           /* sum of the kernels' nE                                  */
    uint32_t n_kernels;
} mcnegf_batch;

int32_t mc_negf_batch_bytes(const mcnegf_kernel* kernels, int32_t n_kernels, uint64_t* bytes_out);
int32_t mc_negf_batch_prepare(const mcnegf_kernel* kernels, int32_t n_kernels,
                              const uint32_t* realizations, uint32_t inject_lead,
                              int64_t* const* d_tallies, void* d_buf, uint64_t buf_bytes,
                              mcnegf_batch* out, hipStream_t stream);
int32_t mc_negf_walk_batch(const mcnegf_batch* b, uint64_t seed, uint64_t walker_begin,
                           uint64_t n_walkers_per_energy, uint32_t max_steps,
                           const mcnegf_walk_config* cfg, hipStream_t stream);
int32_t mc_negf_walk_batch_autotune(const mcnegf_batch* b, uint64_t seed,
                                    uint64_t n_walkers_per_energy, uint32_t max_steps,
                                    mcnegf_walk_config* best, float* best_ms,
                                    hipStream_t stream);

/*
 * Memory-bounded schedule of many systems (host only, no GPU work): assign each of the n
 * systems (nE energies each) to a wave so that the build workspaces of one wave (as
 * mc_negf_workspace_bytes gives them, with each system's flags) fit in budget_bytes.  Systems
 * are taken in decreasing order of their N^2 W cost and put into the first wave with room
 * (first-fit decreasing), so every wave starts with its largest systems; order[k] is the k-th
 * system in that order, wave_of[i] the wave of system i, *n_waves the number of waves.
 * Errors: MCNEGF_EINVAL (bad system, n < 1), MCNEGF_EWS (one system alone exceeds the budget).
 */
int32_t mc_negf_plan_waves(const mcnegf_system* systems, int32_t n, int32_t nE,
                           uint64_t budget_bytes, int32_t* order, int32_t* wave_of,
                           int32_t* n_waves);

/*
 * HIP graph capture of this library's calls (and any other work) on a non-default stream:
 * mc_negf_graph_begin starts capturing `stream`; mc_negf_graph_end stops it and instantiates
 * the graph into *out (a host handle, freed by mc_negf_graph_destroy); mc_negf_graph_launch
 * replays it on `stream`.  Between begin and end only asynchronous calls may be made
 * (mc_negf_build_kernel, mc_negf_walk, mc_negf_walk_batch, mc_negf_walk_sampled,
 * mc_negf_current_async, mc_negf_energy_table, mc_negf_walk_inelastic, mc_negf_spectrum,
 * mc_negf_weighted_tables, mc_negf_walk_weighted, mc_negf_interp_distances,
 * mc_negf_walk_interp; each has a replay test): the synchronising calls fail inside a
 * capture.  No launch timing while capturing.
 */
typedef struct mcnegf_graph_s* mcnegf_graph;
int32_t mc_negf_graph_begin(hipStream_t stream);
int32_t mc_negf_graph_end(hipStream_t stream, mcnegf_graph* out);
int32_t mc_negf_graph_launch(mcnegf_graph g, hipStream_t stream);
int32_t mc_negf_graph_destroy(mcnegf_graph g);

/*
 * Per-launch timing (opt-in, for benchmarks).  Between mc_negf_profile_begin(p) and
 * mc_negf_profile_end(p, ...), every kernel launched by this library from the calling thread
 * is bracketed by two HIP events recorded on the launch stream; p (caller-owned) holds the
 * events and the kernel names.  At most MCNEGF_PROFILE_MAX launches are recorded; later ones
 * are counted in `dropped`.  mc_negf_profile_end synchronises the events, writes each
 * launch's duration in milliseconds to ms_out[0 .. p->n - 1] (host, may be null), destroys
 * the events and detaches p.  Only one profile per thread is active at a time.  Timing never
 * changes a launch's own result: a launch whose events could not be recorded makes
 * mc_negf_profile_end return MCNEGF_EHIP (its duration reads 0).
 */
#define MCNEGF_PROFILE_MAX 512
typedef struct mcnegf_profile {
    int32_t     n;                            /* launches recorded                      */
    int32_t     dropped;                      /* launches beyond MCNEGF_PROFILE_MAX     */
    const char* name[MCNEGF_PROFILE_MAX];     /* static kernel names                    */
    hipEvent_t  start[MCNEGF_PROFILE_MAX];
    hipEvent_t  stop[MCNEGF_PROFILE_MAX];
} mcnegf_profile;

int32_t mc_negf_profile_begin(mcnegf_profile* p);
int32_t mc_negf_profile_end(mcnegf_profile* p, float* ms_out);

/* Synchronise `stream` and copy the device status word to *h_flags. */
int32_t mc_negf_status(const mcnegf_kernel* k, uint32_t* h_flags, hipStream_t stream);

/* The hipError_t of the last failed HIP call in this thread (0 if none). */
int32_t mc_negf_last_hip_error(void);

/* Library version as an integer (major * 10000 + minor * 100 + patch). */
int32_t mc_negf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MCNEGF_H */
