// Gradient of the Monte Carlo transmission estimator by the score function: the derivative of
// the reweighted path estimator of Eq. (66) (Sec. V A, "Improved estimator": walks drawn at
// the current parameters, reweighted by their likelihood ratio at perturbed ones).
//
// A walk injected at lead p scores c_p [exit at q]; with C[o][s] the number of steps s -> o
// of the walks that reached q among N_w walks, p(s -> o) = K_so / S_s (S_s = A_ss for a probe,
// c_p for the injection row, whose normaliser cancels the derivative of c_p), the estimate of
// dT/dtheta is (c_p / N_w) dF/dtheta at fixed counts with
//   F = sum_so C_so K_so / K_so(0) - sum_{s probe} n_s A_ss / A_ss(0),  n_s = sum_o C_so.
// As in the DIRECT adjoint, dF = Re sum_ab Psi_ab dG_ab plus explicit gamma terms:
//   probe s -> probe o:  K = gamma_o |G_so|^2        Psi_so += 2 C_so / G_so
//   A_ss = -2 Im G_ss:                                Psi_ss += -2i n_s / A_ss
//   probe s -> lead q:   K = <G_{:,s}|Gamma_q|G_{:,s}>  Psi_bs += 2 kq_s (Gamma_q conj(G_{sq,s}))_b
//   injection -> probe o: K = gamma_o w_p(o)          Psi_bo += 2 kp_o (Gamma_p conj(G_{sp,o}))_b
//   injection -> lead q: K = T_qp                    Psi_ab += 2 (C_pq / T_qp) (Gamma_p G_qp^+ Gamma_q)_ba
// with kq_s = C_{s->q} / w_q(s), kp_o = C_{p->o} / w_p(o), b in the lead's slice; the explicit
// gamma_o terms add (number of steps into o) / gamma_o.  dG = G dV G (Eq. (7)) and G = G^T give
// dF/dV_m = Re (G Psi G)_mm and dF/dgamma_m = Im (G Psi G)_mm / 2 + explicit.
//
// (G Psi G)_mm = sum_s G_ms (Psi G)_sm and row s of Psi G is (A^{-1} psi_s)^T for psi_s = row s
// of Psi (A = E - H - Sigma symmetric): one block-tridiagonal solve per row with the stored
// left-connected blocks, forward y_k = gL_k (psi_k - t y_{k-1}), backward z_k = y_k - t gL_k z_{k+1},
// O(N W) each; the contributions G_ms z_m of all rows s are summed across the wavefront for
// every m and stored per wavefront.  The lead rows are instead written as
//   sum_b G_mb Psi_bj G_jm = 2 sum_a (G_{m,s} Gamma)_a R_am,  R_a = A^{-1} (k o conj(G_{:,s_a})),
// 2W more solves (lanes N .. N + 2W - 1), assembled per site with the T_qp block.
#include "common.h"

namespace mcnegf {

typedef __attribute__((address_space(3))) double lds_double;

// out = M in for a W x W complex block M (row-major (re, im) pairs in LDS, one address for
// every lane).
template <int W>
__device__ inline void block_matvec(double2 (&out)[W], const double2 (&in)[W], const lds_double* M) {
#pragma unroll
    for (int y = 0; y < W; ++y) {
        double2 acc = cmk(0.0, 0.0);
#pragma unroll
        for (int x = 0; x < W; ++x) cfma(acc, cmk(M[2 * (y * W + x)], M[2 * (y * W + x) + 1]), in[x]);
        out[y] = acc;
    }
}

// Per energy: mu_s = n_s / A_ss (n_s = steps out of probe s, a column sum of the
// outcome-major counts: threads over s read each row coalesced) into sv[0] ([chunk][2][ld]).
__global__ void __launch_bounds__(256) score_prep_kernel(const uint32_t* __restrict__ counts,
                                                         const double* __restrict__ Adiag, int N,
                                                         int64_t ld, double* __restrict__ sv) {
    const int e = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int n = N + 2;
    const uint32_t* C = counts + (size_t)e * n * n;
    uint64_t out = 0;
    for (int o = 0; o < n; ++o) out += C[(size_t)o * n + i];
    const double a = Adiag[(size_t)e * N + i];
    sv[(size_t)e * 2 * ld + i] = out ? (double)out / a : 0.0;
}

// Per energy: the steps into probe o (a row sum of the counts) into sv[1]; one wavefront per
// row, lanes striding along it.
__global__ void __launch_bounds__(64) score_rowsum_kernel(const uint32_t* __restrict__ counts,
                                                          int N, int64_t ld,
                                                          double* __restrict__ sv) {
    const int e = blockIdx.y;
    const int o = blockIdx.x;
    const int n = N + 2;
    const uint32_t* row = counts + (size_t)e * n * n + (size_t)o * n;
    uint64_t in = 0;
    for (int s = threadIdx.x; s < n; s += 64) in += row[s];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) in += __shfl_xor(in, d, 64);
    if (threadIdx.x == 0) sv[(size_t)e * 2 * ld + ld + o] = (double)in;
}

// One lane per right-hand side: c < N is row c of Psi (its probe entries and the diagonal
// term); c = N + a is the solve for R_a of lead p (a < W) or of lead q (a >= W).  The forward
// sweep keeps y in Y[.][c]; the backward sweep stores z only for the lead rows, and the
// wavefront sums G_mc z_m over its lanes c < N for every m, storing the sum in column 64 *
// blockIdx.x of Y (lane 0's own column, whose y at row m it has already read).
template <int W>
__global__ void __launch_bounds__(64) score_solve_kernel(
    const double2* __restrict__ gL, const double2* __restrict__ Gc,
    const uint32_t* __restrict__ counts, const double* __restrict__ sv,
    const double* __restrict__ wL, const double* __restrict__ wR, int L, double t, int64_t ld,
    int64_t ldY, uint32_t inject_lead, double2* __restrict__ Y) {
    const int N = W * L;
    const int n = N + 2;
    const int NC = N + 2 * W;
    const int e = blockIdx.y;
    __shared__ double Ms_raw[2 * 2 * W * W];
    const int tid = threadIdx.x;
    const int c = blockIdx.x * 64 + tid;
    const bool valid = c < NC;
    const bool dense = c < N;
    const bool leadp = valid && !dense && c < N + W;
    const int sp = inject_lead == 0 ? 0 : (L - 1) * W;
    const int sq = inject_lead == 0 ? (L - 1) * W : 0;
    const int pr = N + (int)inject_lead;        // injection row
    const int qo = N + 1 - (int)inject_lead;    // collecting lead
    // the column of G whose entries form this lane's right-hand side
    const int col = dense ? c : (valid ? (leadp ? sp + (c - N) : sq + (c - N - W)) : 0);
    const int cl = valid ? c : 0;  // column of Y that idle lanes read
    const bool has_dense = blockIdx.x * 64 < N;
    const double2* Ge = Gc + (size_t)e * N * ld;
    double2* Ye = Y + (size_t)e * N * ldY;
    const uint32_t* Ce = counts + (size_t)e * n * n;
    const double* wp = (inject_lead == 0 ? wL : wR) + (size_t)e * N;
    const double* wq = (inject_lead == 0 ? wR : wL) + (size_t)e * N;
    const double mu = dense ? sv[(size_t)e * 2 * ld + c] : 0.0;
    const double2* gLe = gL + (size_t)e * L * W * W;
    lds_double* Ms = (lds_double*)Ms_raw;
    constexpr int BS = 2 * W * W;
    auto stage = [&](int buf, int slice) {
#pragma unroll
        for (int i = tid; i < W * W; i += 64) {
            const double2 v = gLe[(size_t)slice * W * W + i];
            Ms[buf * BS + 2 * i] = v.x;
            Ms[buf * BS + 2 * i + 1] = v.y;
        }
    };
    double2 y[W], z[W];
#pragma unroll
    for (int r = 0; r < W; ++r) y[r] = cmk(0.0, 0.0);
    stage(0, 0);
    for (int k = 0; k < L; ++k) {
        __syncthreads();
        const lds_double* cur = Ms + (k & 1) * BS;
        if (k + 1 < L) stage((k + 1) & 1, k + 1);
#pragma unroll
        for (int r = 0; r < W; ++r) {
            const int j = k * W + r;
            const double2 g = Ge[(size_t)j * ld + col];  // G_{j,col} = G_{col,j}
            double2 v;
            if (dense) {
                // 2 C[j][c] / G_cj, and -2i mu_c on the diagonal
                const uint32_t cn = Ce[(size_t)j * n + c];
                const double inv = cn ? 2.0 * (double)cn / cabs2(g) : 0.0;
                v = cmk(inv * g.x, -inv * g.y);
                if (j == c) v.y -= 2.0 * mu;
            } else {
                // k_j conj(G_{j,s_a}): k_j = C[j][pr] / w_p(j) (lead p) or C[qo][j] / w_q(j)
                const uint32_t cn = leadp ? Ce[(size_t)j * n + pr] : Ce[(size_t)qo * n + j];
                const double w = leadp ? wp[j] : wq[j];
                const double kk = (valid && cn) ? (double)cn / w : 0.0;
                v = cmk(kk * g.x, -kk * g.y);
            }
            z[r] = cmk(v.x - t * y[r].x, v.y - t * y[r].y);
        }
        block_matvec<W>(y, z, cur);
        if (valid) {
#pragma unroll
            for (int r = 0; r < W; ++r) Ye[(size_t)(k * W + r) * ldY + c] = y[r];
        }
    }
    // backward: y holds y_{L-1} = z_{L-1}
    __syncthreads();
    if (L > 1) stage(0, L - 2);
    for (int k = L - 1; k >= 0; --k) {
        if (k < L - 1) {
            const int j = L - 2 - k;
            __syncthreads();
            const lds_double* cur = Ms + (j & 1) * BS;
            if (k > 0) stage((j + 1) & 1, k - 1);
            block_matvec<W>(z, y, cur);
#pragma unroll
            for (int r = 0; r < W; ++r) {
                const double2 yk = Ye[(size_t)(k * W + r) * ldY + cl];
                y[r] = cmk(fma(-t, z[r].x, yk.x), fma(-t, z[r].y, yk.y));
            }
        }
        if (valid && !dense) {
#pragma unroll
            for (int r = 0; r < W; ++r) Ye[(size_t)(k * W + r) * ldY + c] = y[r];
        }
        if (has_dense) {  // uniform: the wavefront's sums over its right-hand sides c < N
#pragma unroll
            for (int r = 0; r < W; ++r) {
                const int m = k * W + r;
                double2 v = cmk(0.0, 0.0);
                if (dense) v = cmul(Ge[(size_t)m * ld + c], y[r]);
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) {
                    v.x += __shfl_xor(v.x, o, 64);
                    v.y += __shfl_xor(v.y, o, 64);
                }
                if (tid == 0) Ye[(size_t)m * ldY + 64 * blockIdx.x] = v;
            }
        }
    }
}

// Per energy and site m: (G Psi G)_mm from the wavefront sums and the lead solves, the T_qp
// block, the explicit gamma term, times c_p / N_w.
template <int W>
__global__ void __launch_bounds__(256) score_assemble_kernel(
    const double2* __restrict__ Gc, const double2* __restrict__ Y,
    const uint32_t* __restrict__ counts, const int64_t* __restrict__ tallies,
    const double* __restrict__ sv, const double* __restrict__ gamma,
    const double* __restrict__ lead, const double* __restrict__ gam_lead,
    const double2* __restrict__ corner, int L, int64_t ld, int64_t ldY, uint32_t inject_lead,
    double* __restrict__ gV, double* __restrict__ gG) {
    constexpr int WW = W * W;
    __shared__ double2 psi5[WW];
    const int N = W * L;
    const int n = N + 2;
    const int e = blockIdx.y;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const int sp = inject_lead == 0 ? 0 : (L - 1) * W;
    const int sq = inject_lead == 0 ? (L - 1) * W : 0;
    const int pr = N + (int)inject_lead;
    const int qo = N + 1 - (int)inject_lead;
    const double* gm = gam_lead + (size_t)e * WW;  // Gamma_p = Gamma_q (identical leads)
    const double2* Cq = corner + (size_t)e * 2 * WW + (inject_lead == 0 ? 0 : WW);  // G_{q,p}
    const double* le = lead + (size_t)e * MCNEGF_LEAD_NTERMS;
    const double Tqp = le[inject_lead == 0 ? MCNEGF_LEAD_TRL : MCNEGF_LEAD_TLR];
    const uint32_t cpq = counts[(size_t)e * n * n + (size_t)qo * n + pr];
    const double lpq = (cpq && Tqp > 0.0) ? (double)cpq / Tqp : 0.0;
    for (int tt = threadIdx.x; tt < WW; tt += blockDim.x) {
        const int a = tt / W, b = tt % W;
        // 2 lpq (Gamma_p Cq^+ Gamma_q)[b][a]
        double2 acc = cmk(0.0, 0.0);
        for (int c2 = 0; c2 < W; ++c2)
            for (int d = 0; d < W; ++d) {
                const double f = 2.0 * lpq * gm[b * W + c2] * gm[d * W + a];
                const double2 cc = Cq[d * W + c2];
                acc = cadd(acc, cmk(f * cc.x, -f * cc.y));
            }
        psi5[tt] = acc;
    }
    __syncthreads();
    if (m >= N) return;
    const double2* Ge = Gc + (size_t)e * N * ld;
    const double2* Ym = Y + ((size_t)e * N + m) * ldY;
    double2 K = cmk(0.0, 0.0);
    const int waves = (N + 63) / 64;
    for (int w = 0; w < waves; ++w) K = cadd(K, Ym[64 * w]);
    // lead rows: 2 sum_a (G_{m,s} Gamma)_a R_{a,m}
    double2 gpm[W], gqm[W];
#pragma unroll
    for (int c2 = 0; c2 < W; ++c2) {
        gpm[c2] = Ge[(size_t)(sp + c2) * ld + m];
        gqm[c2] = Ge[(size_t)(sq + c2) * ld + m];
    }
#pragma unroll 1
    for (int a = 0; a < W; ++a) {
        double2 tp = cmk(0.0, 0.0), tq = cmk(0.0, 0.0);
#pragma unroll
        for (int b = 0; b < W; ++b) {
            tp = cadd(tp, cscale(gpm[b], gm[b * W + a]));
            tq = cadd(tq, cscale(gqm[b], gm[b * W + a]));
        }
        K = cadd(K, cscale(cadd(cmul(tp, Ym[N + a]), cmul(tq, Ym[N + W + a])), 2.0));
    }
    // T_qp block: sum_{a in q, b in p} G_ma psi5_ab G_bm
#pragma unroll 1
    for (int a = 0; a < W; ++a) {
        double2 s = cmk(0.0, 0.0);
#pragma unroll
        for (int b = 0; b < W; ++b) s = cadd(s, cmul(psi5[a * W + b], gpm[b]));
        K = cadd(K, cmul(gqm[a], s));
    }
    const int64_t* te = tallies + (size_t)e * MCNEGF_TALLY_N;
    const double walkers =
        (double)(te[MCNEGF_TALLY_EXIT_L] + te[MCNEGF_TALLY_EXIT_R] + te[MCNEGF_TALLY_TRUNC]);
    const double cp = le[inject_lead == 0 ? MCNEGF_LEAD_CL : MCNEGF_LEAD_CR];
    const double scale = walkers > 0.0 ? cp / walkers : 0.0;
    const double g = gamma[m];
    const double in = sv[(size_t)e * 2 * ld + ld + m];
    gV[(size_t)e * N + m] = scale * K.x;
    gG[(size_t)e * N + m] = scale * (0.5 * K.y + (g > 0.0 ? in / g : 0.0));
}

template <int W>
static hipError_t launch_score_w(const mcnegf_kernel& k, const GradBuffers& gb,
                                 const uint32_t* counts, const int64_t* tallies,
                                 uint32_t inject_lead, hipStream_t s) {
    {
        MCNEGF_TIMED("score_prep_kernel", s);
        hipLaunchKernelGGL(score_prep_kernel, dim3((k.N + 255) / 256, k.nE), dim3(256), 0, s,
                           counts, k.Adiag, k.N, gb.ld, gb.xl);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    {
        MCNEGF_TIMED("score_rowsum_kernel", s);
        hipLaunchKernelGGL(score_rowsum_kernel, dim3(k.N, k.nE), dim3(64), 0, s, counts, k.N,
                           gb.ld, gb.xl);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    {
        MCNEGF_TIMED("score_solve_kernel", s);
        hipLaunchKernelGGL(score_solve_kernel<W>, dim3((k.N + 2 * W + 63) / 64, k.nE), dim3(64),
                           0, s, reinterpret_cast<const double2*>(k.gL), gb.G, counts, gb.xl,
                           k.wL, k.wR, k.L, k.t, gb.ld, gb.ldY, inject_lead, gb.Y);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    {
        MCNEGF_TIMED("score_assemble_kernel", s);
        hipLaunchKernelGGL(score_assemble_kernel<W>, dim3((k.N + 255) / 256, k.nE), dim3(256),
                           0, s, gb.G, gb.Y, counts, tallies, gb.xl, k.gamma, k.lead,
                           k.gam_lead, reinterpret_cast<const double2*>(k.corner), k.L, gb.ld,
                           gb.ldY, inject_lead, gb.gV, gb.gG);
    }
    return hipGetLastError();
}

hipError_t launch_score_grad(const mcnegf_kernel& k, const GradBuffers& gb,
                             const uint32_t* counts, const int64_t* tallies,
                             uint32_t inject_lead, const double* weights, double* dI_dV,
                             double* dI_dgamma, int chunk, hipStream_t s) {
    const int N = k.N, nE = k.nE;
    const size_t n = (size_t)k.n_out;
    hipError_t err;
    for (int e0 = 0; e0 < nE; e0 += chunk) {
        const int nc = min(chunk, nE - e0);
        const mcnegf_kernel kc = energy_slice(k, e0, nc);
        GradBuffers g = gb;
        g.gV = gb.gV + (size_t)e0 * N;
        g.gG = gb.gG + (size_t)e0 * N;
        const uint32_t* ce = counts + (size_t)e0 * n * n;
        const int64_t* te = tallies + (size_t)e0 * MCNEGF_TALLY_N;
        if ((err = launch_fullinv_store_g(kc, g.G, g.ld, s)) != hipSuccess) return err;
        switch (k.W) {
#define MCNEGF_CASE(w)                                                                 \
    case w:                                                                            \
        if ((err = launch_score_w<w>(kc, g, ce, te, inject_lead, s)) != hipSuccess)   \
            return err;                                                                \
        break;
            MCNEGF_CASE(1) MCNEGF_CASE(2) MCNEGF_CASE(3) MCNEGF_CASE(4) MCNEGF_CASE(5)
            MCNEGF_CASE(6) MCNEGF_CASE(7) MCNEGF_CASE(8) MCNEGF_CASE(9) MCNEGF_CASE(10)
            MCNEGF_CASE(11) MCNEGF_CASE(12) MCNEGF_CASE(13) MCNEGF_CASE(14) MCNEGF_CASE(15)
            MCNEGF_CASE(16) MCNEGF_CASE(17) MCNEGF_CASE(18) MCNEGF_CASE(19) MCNEGF_CASE(20)
            MCNEGF_CASE(21) MCNEGF_CASE(22) MCNEGF_CASE(23) MCNEGF_CASE(24) MCNEGF_CASE(25)
            MCNEGF_CASE(26) MCNEGF_CASE(27) MCNEGF_CASE(28) MCNEGF_CASE(29) MCNEGF_CASE(30)
            MCNEGF_CASE(31) MCNEGF_CASE(32)
#undef MCNEGF_CASE
            default:
                return hipErrorInvalidValue;
        }
    }
    return launch_grad_reduce(gb, weights, nE, N, dI_dV, dI_dgamma, s);
}

}  // namespace mcnegf
