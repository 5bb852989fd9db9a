// Gradient of the DIRECT current I = sum_k w_k T_k with respect to the onsite potentials V_i
// and the dephasing rates gamma_i (Sigma_s,ii = -(i/2) gamma_i, Sec. III A, Eq. (77)).
//
// With injection from lead p and collection at q (f_p = 1, f_q = 0), Sec. III C, Eq. (79)
// read as the diagonal of Eq. (8):
//   T = T_qp + c^T M^{-1} b,  M = diag(gamma_j A_jj) - T_PP,  b_j = gamma_j w_p(j),
//   c_j = gamma_j w_q(j),  T_PP,ij = gamma_i gamma_j |G_ij|^2,  A_jj = -2 Im G_jj,
//   w_r(j) = (G Gamma_r G^+)_jj,  T_qp = Tr Gamma_q G_qp Gamma_p G_qp^+.
// Adjoint: x = M^{-1} b, lambda = M^{-1} c (M is symmetric), u = gamma lambda, v = gamma x.
// At fixed gamma, dT = Re sum_ab Psi_ab dG_ab with
//   Psi_ab   = 2 u_a v_b conj(G_ab)                              (|G_ab|^2 in M)
//   Psi_jj  += -2i u_j x_j                                       (A_jj in M)
//   Psi_ja  += 2 u_j sum_c Gamma_p,ac conj(G_jc),  a, c in slice p   (w_p in b)
//   Psi_ja  += 2 v_j sum_c Gamma_q,ac conj(G_jc),  a, c in slice q   (w_q in c)
//   Psi_ab  += 2 (Gamma_p G_qp^+ Gamma_q)_ba,  a in slice q, b in slice p   (T_qp)
// and dG = G dV G (dA = -dV), so dT/dV_i = Re K_i with K = diag(G Psi G); a change of
// gamma_i changes A by (i/2) e_i e_i^T, giving Im K_i / 2, plus the explicit terms
//   lambda_i w_p(i) + x_i w_q(i) - lambda_i A_ii x_i + lambda_i (P v)_i + x_i (P u)_i.
// G is complex symmetric, so G_ij = G_ji and Q = conj(G) diag(v) G is Hermitian; the dense
// part of K is 2 sum_a G_ia u_a Q_ai, with Q from one batched complex GEMM.
#include <rocblas/rocblas.h>

#include <mutex>

#include "common.h"

namespace mcnegf {

__device__ inline int perm16(int j) { return (j & ~15) + 4 * (j & 3) + ((j >> 2) & 3); }

__device__ inline double readlane_dbl(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// L^T xt = y and L^T lt = z with L the Cholesky factor of the bordered scaled probe system
// (lower part, columns of each 16-block stored permuted) and y, z its bordered rows Np and
// Np + 1; then x = s xt and lambda = s lt (s_j = M_jj^{-1/2}, vector slot 3).  One workgroup
// of 256 threads per energy, block columns of 64 from the last one down: the rows below a
// block contribute by a transposed matrix-vector product (thread = stored column position p
// x row group), the 64 x 64 diagonal block by back substitution in one wavefront.  xt and
// lt are solved in place in xl ([nE][2][ld], the solved entries stay in L2); padded entries
// N..Np-1 are left as solved (zero).
__global__ void __launch_bounds__(256) backsolve_kernel(const double* __restrict__ Lall,
                                                        const double* __restrict__ vec, int N,
                                                        int Np, int64_t ld,
                                                        double* __restrict__ xl) {
    __shared__ double part[4][64][2];
    const int e = blockIdx.x;
    double* sol = xl + (size_t)e * 2 * ld;  // [0, Np): xt, [ld, ld + Np): lt
    const int tid = threadIdx.x;
    const int p = tid & 63, grp = tid >> 6;
    const int R = Np + 2;
    const double* Le = Lall + (size_t)e * R * ld;
    const int nJ = (Np + 63) / 64;
    for (int J = nJ - 1; J >= 0; --J) {
        const int c0 = 64 * J;
        const int wJ = min(64, Np - c0);
        double sx = 0.0, sl = 0.0;
        if (p < wJ) {
            for (int i = c0 + wJ + grp; i < Np; i += 4) {
                const double lij = Le[(size_t)i * ld + c0 + p];
                sx = fma(lij, sol[i], sx);
                sl = fma(lij, sol[ld + i], sl);
            }
        }
        part[grp][p][0] = sx;
        part[grp][p][1] = sl;
        __syncthreads();
        if (grp == 0) {
            // lane m: logical column m of the block, stored at position perm16(m)
            const int m = tid;
            const int pm = perm16(m);
            double rx = 0.0, rl = 0.0;
            if (m < wJ) {
                rx = Le[(size_t)Np * ld + c0 + pm] -
                     (part[0][pm][0] + part[1][pm][0] + part[2][pm][0] + part[3][pm][0]);
                rl = Le[(size_t)(Np + 1) * ld + c0 + pm] -
                     (part[0][pm][1] + part[1][pm][1] + part[2][pm][1] + part[3][pm][1]);
            }
            for (int k = wJ - 1; k >= 0; --k) {  // uniform loop, whole wavefront active
                const double lkk = Le[(size_t)(c0 + k) * ld + c0 + perm16(k)];
                const double xk = readlane_dbl(rx, k) / lkk;
                const double lk = readlane_dbl(rl, k) / lkk;
                const double lkm = (m < k) ? Le[(size_t)(c0 + k) * ld + c0 + pm] : 0.0;
                rx = (m == k) ? xk : fma(-lkm, xk, rx);
                rl = (m == k) ? lk : fma(-lkm, lk, rl);
            }
            if (m < wJ) {
                sol[c0 + m] = rx;
                sol[ld + c0 + m] = rl;
            }
        }
        __syncthreads();
    }
    const double* s = vec + (size_t)e * 4 * N + 3 * N;
    for (int j = tid; j < N; j += 256) {  // each entry read and written by one thread
        sol[j] *= s[j];
        sol[ld + j] *= s[j];
    }
}

// H[i][b] = G[i][b] v_b with v = gamma x (row-major, pitch ld; columns < N).
__global__ void grad_scale_kernel(const double2* __restrict__ Gc, const double* __restrict__ xl,
                                  const double* __restrict__ gamma, int N, int64_t ld,
                                  double2* __restrict__ H) {
    const int e = blockIdx.z;
    const int i = blockIdx.y;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= N) return;
    const double vb = gamma[b] * xl[(size_t)e * 2 * ld + b];
    const size_t at = ((size_t)e * N + i) * ld + b;
    const double2 g = Gc[at];
    H[at] = cmk(g.x * vb, g.y * vb);
}

// Per energy and row i: K_i and the explicit gamma terms (see the top of the file).
// Threads run over i, the loop over j reads G[j][i] = G_ij and Q_mem[j][i] = Q_ij (both
// coalesced) and the slice entries G[j][sp..], G[j][sq..] (uniform).
template <int W>
__global__ void __launch_bounds__(256) grad_assemble_kernel(
    const double2* __restrict__ Gc, const double2* __restrict__ Q, const double* __restrict__ xl,
    const double* __restrict__ gamma, const double* __restrict__ wL, const double* __restrict__ wR,
    const double* __restrict__ Adiag, const double* __restrict__ gam_lead,
    const double2* __restrict__ corner, int L, int64_t ld, uint32_t inject_lead,
    double* __restrict__ gV, double* __restrict__ gG) {
    constexpr int WW = W * W;
    __shared__ double2 psi5[WW];  // Psi5[a][b], a in slice q, b in slice p
    const int N = W * L;
    const int e = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int sp = inject_lead == 0 ? 0 : (L - 1) * W;  // first site of slice p
    const int sq = inject_lead == 0 ? (L - 1) * W : 0;  // first site of slice q
    const double* gm = gam_lead + (size_t)e * WW;       // Gamma_p = Gamma_q (identical leads)
    // corner C = G_{q,p}: G_{L-1,0} for injection from L, G_{0,L-1} from R
    const double2* C = corner + (size_t)e * 2 * WW + (inject_lead == 0 ? 0 : WW);
    for (int t = threadIdx.x; t < WW; t += blockDim.x) {
        const int a = t / W, b = t % W;
        // Psi5[a][b] = 2 (Gamma_p C^+ Gamma_q)[b][a] = 2 sum_{c,d} Gp[b][c] conj(C[d][c]) Gq[d][a]
        double2 acc = cmk(0.0, 0.0);
        for (int c = 0; c < W; ++c)
            for (int d = 0; d < W; ++d) {
                const double f = 2.0 * gm[b * W + c] * gm[d * W + a];
                const double2 cc = C[d * W + c];
                acc = cadd(acc, cmk(f * cc.x, -f * cc.y));
            }
        psi5[t] = acc;
    }
    __syncthreads();
    if (i >= N) return;
    const double2* Ge = Gc + (size_t)e * N * ld;
    const double2* Qe = Q + (size_t)e * N * ld;
    const double* xe = xl + (size_t)e * 2 * ld;
    const double* le = xe + ld;
    double2 kd = cmk(0.0, 0.0), kg = cmk(0.0, 0.0);
    double2 al[W], be[W];
#pragma unroll
    for (int b = 0; b < W; ++b) {
        al[b] = cmk(0.0, 0.0);
        be[b] = cmk(0.0, 0.0);
    }
    double pv = 0.0, pu = 0.0;
    for (int j = 0; j < N; ++j) {
        const double2 gij = Ge[(size_t)j * ld + i];
        const double2 qji = Qe[(size_t)j * ld + i];  // Q_mem[j][i] = Q_ij; Q_ji = conj(Q_ij)
        const double gj = gamma[j];
        const double uj = gj * le[j], vj = gj * xe[j];
        // dense: G_ij u_j Q_ji
        const double2 gu = cscale(gij, uj);
        kd = cadd(kd, cmul(gu, cconj(qji)));
        // diagonal: G_ij^2 u_j x_j
        kg = cadd(kg, cscale(cmul(gij, gij), uj * xe[j]));
        const double pij = cabs2(gij);
        pv = fma(pij, vj, pv);
        pu = fma(pij, uj, pu);
        const double2 gv = cscale(gij, vj);
#pragma unroll
        for (int b = 0; b < W; ++b) {
            al[b] = cadd(al[b], cmul(gu, cconj(Ge[(size_t)j * ld + sp + b])));
            be[b] = cadd(be[b], cmul(gv, cconj(Ge[(size_t)j * ld + sq + b])));
        }
    }
    double2 K = cadd(cscale(kd, 2.0), cmk(2.0 * kg.y, -2.0 * kg.x));  // 2 kd - 2i kg
    // lead terms: 2 sum_b al_b (Gamma_p G_{p,i})_b + 2 sum_b be_b (Gamma_q G_{q,i})_b
    double2 gpi[W], gqi[W];
#pragma unroll
    for (int c = 0; c < W; ++c) {
        gpi[c] = Ge[(size_t)(sp + c) * ld + i];
        gqi[c] = Ge[(size_t)(sq + c) * ld + i];
    }
#pragma unroll
    for (int b = 0; b < W; ++b) {
        double2 tp = cmk(0.0, 0.0), tq = cmk(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < W; ++c) {
            tp = cadd(tp, cscale(gpi[c], gm[b * W + c]));
            tq = cadd(tq, cscale(gqi[c], gm[b * W + c]));
        }
        K = cadd(K, cscale(cadd(cmul(al[b], tp), cmul(be[b], tq)), 2.0));
    }
    // T_qp term: sum_{a in q, b in p} G_ia Psi5_ab G_bi
#pragma unroll
    for (int a = 0; a < W; ++a) {
        double2 s = cmk(0.0, 0.0);
#pragma unroll
        for (int b = 0; b < W; ++b) s = cadd(s, cmul(psi5[a * W + b], gpi[b]));
        K = cadd(K, cmul(gqi[a], s));
    }
    const double wp = inject_lead == 0 ? wL[(size_t)e * N + i] : wR[(size_t)e * N + i];
    const double wq = inject_lead == 0 ? wR[(size_t)e * N + i] : wL[(size_t)e * N + i];
    const double Aii = Adiag[(size_t)e * N + i];
    double lam = le[i], x = xe[i];
    if (gamma[i] == 0.0) {
        // The site is absent from the probe system (its row of M vanishes), but x_i and
        // lambda_i have finite limits as gamma_i -> 0: row i of M x = b divided by gamma_i.
        x = (wp + pv) / Aii;
        lam = (wq + pu) / Aii;
    }
    gV[(size_t)e * N + i] = K.x;
    gG[(size_t)e * N + i] = 0.5 * K.y + lam * wp + x * wq - lam * Aii * x + lam * pv + x * pu;
}

// dI/dV_i = sum_k w_k gV[k][i], dI/dgamma_i likewise (fixed order over k).
__global__ void grad_reduce_kernel(const double* __restrict__ gV, const double* __restrict__ gG,
                                   const double* __restrict__ w, int nE, int N,
                                   double* __restrict__ dV, double* __restrict__ dG) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < nE; ++k) {
        a = fma(w[k], gV[(size_t)k * N + i], a);
        b = fma(w[k], gG[(size_t)k * N + i], b);
    }
    dV[i] = a;
    dG[i] = b;
}

static rocblas_handle blas_handle(hipError_t& err) {
    static std::mutex mu;
    static rocblas_handle handles[64] = {};
    int dev = 0;
    if ((err = hipGetDevice(&dev)) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!handles[dev] && rocblas_create_handle(&handles[dev]) != rocblas_status_success)
        handles[dev] = nullptr;
    if (!handles[dev]) err = hipErrorNotInitialized;
    return handles[dev];
}

template <int W>
static hipError_t launch_assemble_w(const mcnegf_kernel& k, const GradBuffers& gb,
                                    uint32_t inject_lead, hipStream_t s) {
    {
        MCNEGF_TIMED("grad_assemble_kernel", s);
        hipLaunchKernelGGL(grad_assemble_kernel<W>, dim3((k.N + 255) / 256, k.nE), dim3(256), 0,
                           s, gb.G, gb.Q, gb.xl, k.gamma, k.wL, k.wR, k.Adiag, k.gam_lead,
                           reinterpret_cast<const double2*>(k.corner), k.L, gb.ld, inject_lead,
                           gb.gV, gb.gG);
    }
    return hipGetLastError();
}

hipError_t launch_grad(const mcnegf_kernel& k, const GradBuffers& gb, uint32_t inject_lead,
                       const double* weights, double* dI_dV, double* dI_dgamma, hipStream_t s) {
    const int N = k.N, nE = k.nE;
    const int Np = (int)k.p_pitch;
    hipError_t err;
    {
        MCNEGF_TIMED("backsolve_kernel", s);
        hipLaunchKernelGGL(backsolve_kernel, dim3(nE), dim3(256), 0, s, k.direct, k.direct_vec,
                           N, Np, k.p_pitch, gb.xl);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    if ((err = launch_fullinv_store_g(k, gb.G, gb.ld, s)) != hipSuccess) return err;
    {
        MCNEGF_TIMED("grad_scale_kernel", s);
        hipLaunchKernelGGL(grad_scale_kernel, dim3((N + 255) / 256, N, nE), dim3(256), 0, s, gb.G,
                           gb.xl, k.gamma, N, gb.ld, gb.H);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    {
        // Q = conj(G) H in column-major terms: the row-major arrays of the symmetric G and of
        // H read column-major are G and diag(v) G; op C on G gives G^+ = conj(G); Q lands as
        // Q_mem[i][a] = Q_ai.
        rocblas_handle h = blas_handle(err);
        if (!h) return err;
        if (rocblas_set_stream(h, s) != rocblas_status_success) return hipErrorInvalidValue;
        const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
        const rocblas_stride st = (rocblas_stride)N * gb.ld;
        MCNEGF_TIMED("grad_zgemm", s);
        const rocblas_status rs = rocblas_zgemm_strided_batched(
            h, rocblas_operation_conjugate_transpose, rocblas_operation_none, N, N, N, &one,
            reinterpret_cast<const rocblas_double_complex*>(gb.G), (rocblas_int)gb.ld, st,
            reinterpret_cast<const rocblas_double_complex*>(gb.H), (rocblas_int)gb.ld, st, &zero,
            reinterpret_cast<rocblas_double_complex*>(gb.Q), (rocblas_int)gb.ld, st, nE);
        if (rs != rocblas_status_success) return hipErrorLaunchFailure;
    }
    switch (k.W) {
#define MCNEGF_CASE(w)                                                         \
    case w:                                                                    \
        if ((err = launch_assemble_w<w>(k, gb, inject_lead, s)) != hipSuccess) \
            return err;                                                        \
        break;
        MCNEGF_CASE(1) MCNEGF_CASE(2) MCNEGF_CASE(3) MCNEGF_CASE(4) MCNEGF_CASE(5)
        MCNEGF_CASE(6) MCNEGF_CASE(7) MCNEGF_CASE(8) MCNEGF_CASE(9) MCNEGF_CASE(10)
        MCNEGF_CASE(11) MCNEGF_CASE(12) MCNEGF_CASE(13) MCNEGF_CASE(14) MCNEGF_CASE(15)
        MCNEGF_CASE(16)
#undef MCNEGF_CASE
        default:
            return hipErrorInvalidValue;
    }
    {
        MCNEGF_TIMED("grad_reduce_kernel", s);
        hipLaunchKernelGGL(grad_reduce_kernel, dim3((N + 255) / 256), dim3(256), 0, s, gb.gV,
                           gb.gG, weights, nE, N, dI_dV, dI_dgamma);
    }
    return hipGetLastError();
}

}  // namespace mcnegf
