// Effective transmissions and the current.
//
// MC (Sec. II E, Eq. (66); relative deviation as in Sec. IV A): with injection at lead p,
//   p_k = exits at the other lead q / walkers,  T_k = c_p p_k,
//   sigma_k = c_p sqrt(p_k (1 - p_k) / (walkers - 1)),  c_p = total of injection row p.
// DIRECT (Sec. III C, Eq. (79)): the diagonal of G^< = G Sigma^< G^+ (Eq. (8)) with
// Buttiker lesser self-energies gamma_i n_i gives, per probe j,
//   gamma_j A_jj n_j - sum_i T_ji n_i = T_jp   (f_p = 1, f_q = 0),  T_ji = gamma_j gamma_i |G_ji|^2,
// a symmetric, weakly diagonally dominant system with positive diagonal (its row sums are
// the probe's couplings to the leads), so Cholesky without pivoting applies.  It is solved
// in the symmetrically scaled form S M S with S = diag(M_jj^{-1/2}); probes with
// gamma_j = 0 decouple (identity row).  Then T_k = T_qp + sum_j T_qj n_j.
// Current: I = sum_k w_k T_k (midpoint quadrature, Sec. III C), sigma_I^2 = sum_k w_k^2 sigma_k^2.
#include "common.h"

namespace mcnegf {

__device__ inline double block_reduce256(double v, double* red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Weighted sums over energies (one block, fixed order): out[0] = sum w T, out[1] = sum w^2 s^2.
__global__ void __launch_bounds__(256) current_sum_kernel(const double* __restrict__ T,
                                                          const double* __restrict__ sig,
                                                          const double* __restrict__ w, int nE,
                                                          double* __restrict__ out) {
    __shared__ double red[256];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nE; k += 256) {
        a += w[k] * T[k];
        b += w[k] * w[k] * sig[k] * sig[k];
    }
    a = block_reduce256(a, red);
    b = block_reduce256(b, red);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

__global__ void mc_current_kernel(const int64_t* __restrict__ tallies,
                                  const double* __restrict__ lead, int nE, uint32_t inject_lead,
                                  double* __restrict__ T, double* __restrict__ sig) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nE) return;
    const int64_t* t = tallies + (size_t)k * MCNEGF_TALLY_N;
    const double walkers =
        (double)(t[MCNEGF_TALLY_EXIT_L] + t[MCNEGF_TALLY_EXIT_R] + t[MCNEGF_TALLY_TRUNC]);
    const double hits = (double)(inject_lead == 0 ? t[MCNEGF_TALLY_EXIT_R] : t[MCNEGF_TALLY_EXIT_L]);
    const double c = lead[(size_t)k * MCNEGF_LEAD_NTERMS +
                          (inject_lead == 0 ? MCNEGF_LEAD_CL : MCNEGF_LEAD_CR)];
    if (walkers <= 0.0) {
        T[k] = 0.0;
        sig[k] = 0.0;
        return;
    }
    const double p = hits / walkers;
    T[k] = c * p;
    sig[k] = walkers > 1.0 ? c * sqrt(p * (1.0 - p) / (walkers - 1.0)) : 0.0;
}

hipError_t launch_mc_current(const mcnegf_kernel& k, uint32_t inject_lead, const int64_t* tallies,
                             const double* weights, double* T, double* sigmaT, hipStream_t s) {
    {
        MCNEGF_TIMED("mc_current_kernel", s);
        hipLaunchKernelGGL(mc_current_kernel, dim3((k.nE + 255) / 256), dim3(256), 0, s, tallies,
                           k.lead, k.nE, inject_lead, T, sigmaT);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    {
        MCNEGF_TIMED("current_sum_kernel", s);
        hipLaunchKernelGGL(current_sum_kernel, dim3(1), dim3(256), 0, s, T, sigmaT, weights, k.nE,
                           k.reduce);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- DIRECT
// vec layout per energy: [0] scale s_j, [1] right-hand side (scaled), [2] solution, [3] T_qj
__global__ void direct_prep_kernel(const double* __restrict__ P, const double* __restrict__ Adiag,
                                   const double* __restrict__ wL, const double* __restrict__ wR,
                                   const double* __restrict__ gamma, int N, int64_t ldP,
                                   uint32_t inject_lead, double* __restrict__ vec) {
    const int e = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const double g = gamma[j];
    const double Pjj = P[((size_t)e * N + j) * ldP + j];
    const double mjj = g * Adiag[(size_t)e * N + j] - g * g * Pjj;
    const double sj = (g > 0.0 && mjj > 0.0) ? 1.0 / sqrt(mjj) : 0.0;
    const double wp = inject_lead == 0 ? wL[(size_t)e * N + j] : wR[(size_t)e * N + j];
    const double wq = inject_lead == 0 ? wR[(size_t)e * N + j] : wL[(size_t)e * N + j];
    double* v = vec + (size_t)e * 4 * N;
    v[j] = sj;
    v[N + j] = g * wp * sj;
    v[3 * N + j] = g * wq;
}

__global__ void __launch_bounds__(256) direct_fill_kernel(const double* __restrict__ P,
                                                          const double* __restrict__ gamma,
                                                          const double* __restrict__ vec, int N,
                                                          int64_t ld, double* __restrict__ M) {
    const int e = blockIdx.y;
    const int i = blockIdx.x;
    const double* sv = vec + (size_t)e * 4 * N;
    const double si = sv[i];
    const double gi = gamma[i];
    const double* Pr = P + ((size_t)e * N + i) * ld;
    double* Mr = M + ((size_t)e * N + i) * ld;
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        double m;
        if (si == 0.0 || sv[j] == 0.0) m = (i == j) ? 1.0 : 0.0;
        else if (i == j) m = 1.0;
        else m = -gi * gamma[j] * Pr[j] * si * sv[j];
        Mr[j] = m;
    }
}

constexpr int NB = 32;

// Right-looking blocked Cholesky (lower) of one energy's N x N matrix, one workgroup.
__global__ void __launch_bounds__(256) cholesky_kernel(double* __restrict__ Mall, int N, int64_t ld,
                                                       uint32_t* __restrict__ status) {
    __shared__ double D[NB][NB + 1];
    __shared__ double Pa[NB][NB + 1];
    __shared__ double Pb[NB][NB + 1];
    __shared__ int bad;
    double* A = Mall + (size_t)blockIdx.x * N * ld;
    const int tid = threadIdx.x;
    const int nt = (N + NB - 1) / NB;
    if (tid == 0) bad = 0;
    for (int jb = 0; jb < nt; ++jb) {
        const int j0 = jb * NB;
        const int jn = min(NB, N - j0);
        for (int idx = tid; idx < NB * NB; idx += 256) {
            const int r = idx / NB, c = idx % NB;
            D[r][c] = (r < jn && c < jn) ? A[(size_t)(j0 + r) * ld + j0 + c] : (r == c ? 1.0 : 0.0);
        }
        __syncthreads();
        for (int c = 0; c < NB; ++c) {
            if (tid == 0) {
                double d = D[c][c];
                if (!(d > 0.0)) {
                    bad = 1;
                    d = 1.0;
                }
                D[c][c] = sqrt(d);
            }
            __syncthreads();
            if (tid > c && tid < NB) D[tid][c] /= D[c][c];
            __syncthreads();
            for (int idx = tid; idx < NB * NB; idx += 256) {
                const int r = idx / NB, q = idx % NB;
                if (r > c && q > c && q <= r) D[r][q] -= D[r][c] * D[q][c];
            }
            __syncthreads();
        }
        for (int idx = tid; idx < NB * NB; idx += 256) {
            const int r = idx / NB, c = idx % NB;
            if (r < jn && c < jn && c <= r) A[(size_t)(j0 + r) * ld + j0 + c] = D[r][c];
        }
        // panel below: X D^T = A_panel, one row per thread
        for (int i = j0 + NB + tid; i < N; i += 256) {
            double x[NB];
            double* Ar = A + (size_t)i * ld + j0;
#pragma unroll
            for (int c = 0; c < NB; ++c) x[c] = (c < jn) ? Ar[c] : 0.0;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                x[c] = x[c] / D[c][c];
#pragma unroll
                for (int q = c + 1; q < NB; ++q) x[q] = fma(-x[c], D[q][c], x[q]);
                __asm__ volatile("" ::: "memory");  // keep the LDS reads of column c here
            }
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < jn) Ar[c] = x[c];
        }
        __threadfence_block();
        __syncthreads();
        // trailing update A[ib][kb] -= P_ib P_kb^T for jb < kb <= ib
        const int tr = tid / 16, tc = tid % 16;  // 2x2 outputs per thread
        for (int ib = jb + 1; ib < nt; ++ib) {
            const int i0 = ib * NB;
            const int in_ = min(NB, N - i0);
            for (int idx = tid; idx < NB * NB; idx += 256) {
                const int r = idx / NB, c = idx % NB;
                Pa[r][c] = (r < in_ && c < jn) ? A[(size_t)(i0 + r) * ld + j0 + c] : 0.0;
            }
            for (int kb = jb + 1; kb <= ib; ++kb) {
                const int k0 = kb * NB;
                const int kn = min(NB, N - k0);
                for (int idx = tid; idx < NB * NB; idx += 256) {
                    const int r = idx / NB, c = idx % NB;
                    Pb[r][c] = (r < kn && c < jn) ? A[(size_t)(k0 + r) * ld + j0 + c] : 0.0;
                }
                __syncthreads();
                double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll 8
                for (int q = 0; q < NB; ++q) {
                    const double a0 = Pa[2 * tr][q], a1 = Pa[2 * tr + 1][q];
                    const double b0 = Pb[2 * tc][q], b1 = Pb[2 * tc + 1][q];
                    acc[0][0] = fma(a0, b0, acc[0][0]);
                    acc[0][1] = fma(a0, b1, acc[0][1]);
                    acc[1][0] = fma(a1, b0, acc[1][0]);
                    acc[1][1] = fma(a1, b1, acc[1][1]);
                }
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < 2; ++v) {
                        const int r = 2 * tr + u, c = 2 * tc + v;
                        if (r < in_ && c < kn) A[(size_t)(i0 + r) * ld + k0 + c] -= acc[u][v];
                    }
                __syncthreads();
            }
        }
        __threadfence_block();
        __syncthreads();
    }
    if (tid == 0 && bad) atomicOr(status, MCNEGF_FLAG_NOTSPD);
}

// Forward and backward substitution with the Cholesky factor, then T_k.
__global__ void __launch_bounds__(256) chol_solve_kernel(const double* __restrict__ Mall, int N,
                                                         int64_t ld, double* __restrict__ vec,
                                                         const double* __restrict__ lead,
                                                         uint32_t inject_lead, double* __restrict__ T,
                                                         double* __restrict__ sig,
                                                         uint32_t* __restrict__ status) {
    extern __shared__ double y[];
    __shared__ double red[256];
    const int e = blockIdx.x;
    const double* A = Mall + (size_t)e * N * ld;
    double* v = vec + (size_t)e * 4 * N;
    const int tid = threadIdx.x;
    const int nt = (N + NB - 1) / NB;
    for (int i = tid; i < N; i += 256) y[i] = v[N + i];
    __syncthreads();
    // L y = b
    for (int jb = 0; jb < nt; ++jb) {
        const int j0 = jb * NB, jn = min(NB, N - j0);
        if (tid == 0) {
            for (int c = 0; c < jn; ++c) {
                double acc = y[j0 + c];
                for (int q = 0; q < c; ++q) acc -= A[(size_t)(j0 + c) * ld + j0 + q] * y[j0 + q];
                y[j0 + c] = acc / A[(size_t)(j0 + c) * ld + j0 + c];
            }
        }
        __syncthreads();
        for (int i = j0 + jn + tid; i < N; i += 256) {
            double acc = 0.0;
            for (int q = 0; q < jn; ++q) acc += A[(size_t)i * ld + j0 + q] * y[j0 + q];
            y[i] -= acc;
        }
        __syncthreads();
    }
    // L^T x = y
    for (int jb = nt - 1; jb >= 0; --jb) {
        const int j0 = jb * NB, jn = min(NB, N - j0);
        if (tid == 0) {
            for (int c = jn - 1; c >= 0; --c) {
                double acc = y[j0 + c];
                for (int q = c + 1; q < jn; ++q) acc -= A[(size_t)(j0 + q) * ld + j0 + c] * y[j0 + q];
                y[j0 + c] = acc / A[(size_t)(j0 + c) * ld + j0 + c];
            }
        }
        __syncthreads();
        for (int r = tid; r < j0; r += 256) {
            double acc = 0.0;
            for (int q = 0; q < jn; ++q) acc += A[(size_t)(j0 + q) * ld + r] * y[j0 + q];
            y[r] -= acc;
        }
        __syncthreads();
    }
    // n_j = s_j x_j;  T = T_qp + sum_j T_qj n_j
    double part = 0.0;
    for (int i = tid; i < N; i += 256) {
        const double nj = v[i] * y[i];
        v[2 * N + i] = nj;
        part += v[3 * N + i] * nj;
    }
    const double sum = block_reduce256(part, red);
    if (tid == 0) {
        const double* ld_ = lead + (size_t)e * MCNEGF_LEAD_NTERMS;
        const double tqp = inject_lead == 0 ? ld_[MCNEGF_LEAD_TRL] : ld_[MCNEGF_LEAD_TLR];
        const double Tk = tqp + sum;
        T[e] = Tk;
        sig[e] = 0.0;
        if (!isfinite(Tk)) atomicOr(status, MCNEGF_FLAG_NONFINITE);
    }
}

hipError_t launch_direct_current(const mcnegf_kernel& k, uint32_t inject_lead,
                                 const double* weights, double* T, double* sigmaT, hipStream_t s) {
    const int N = k.N;
    {
        MCNEGF_TIMED("direct_prep_kernel", s);
        hipLaunchKernelGGL(direct_prep_kernel, dim3((N + 255) / 256, k.nE), dim3(256), 0, s, k.P,
                           k.Adiag, k.wL, k.wR, k.gamma, N, k.p_pitch, inject_lead, k.direct_vec);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    {
        MCNEGF_TIMED("direct_fill_kernel", s);
        hipLaunchKernelGGL(direct_fill_kernel, dim3(N, k.nE), dim3(256), 0, s, k.P, k.gamma,
                           k.direct_vec, N, k.p_pitch, k.direct);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    {
        MCNEGF_TIMED("cholesky_kernel", s);
        hipLaunchKernelGGL(cholesky_kernel, dim3(k.nE), dim3(256), 0, s, k.direct, N, k.p_pitch,
                           k.status);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    {
        MCNEGF_TIMED("chol_solve_kernel", s);
        hipLaunchKernelGGL(chol_solve_kernel, dim3(k.nE), dim3(256), (size_t)N * sizeof(double), s,
                           k.direct, N, k.p_pitch, k.direct_vec, k.lead, inject_lead, T, sigmaT,
                           k.status);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    {
        MCNEGF_TIMED("current_sum_kernel", s);
        hipLaunchKernelGGL(current_sum_kernel, dim3(1), dim3(256), 0, s, T, sigmaT, weights, k.nE,
                           k.reduce);
    }
    return hipGetLastError();
}

}  // namespace mcnegf
