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
// G is complex symmetric (G_ij = G_ji), so with Q = conj(G) diag(v) G and R = conj(G) diag(u) G
//   dense part of K_i = 2 sum_a G_ia u_a Q_ai,
//   lead parts:  sum_j G_ij u_j conj(G_{j,sp+b}) = conj(R_{i,sp+b}),
//                sum_j G_ij v_j conj(G_{j,sq+b}) = conj(Q_{i,sq+b}).
// A column of Q or R is conj(A)^{-1} applied to d o G_{:,c} (A = E - H - Sigma, block
// tridiagonal with off-diagonal blocks t I), solved by the block LU of A that the stored
// left-connected blocks gL_k provide:
//   forward   y_k = conj(gL_k) (h_k - t y_{k-1}),   backward  q_k = y_k - t conj(gL_k) q_{k+1},
// O(N W) per column instead of a dense O(N^2) product.
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
// of 1024 threads per energy, right-looking over block rows of 64 from the last one down:
//   solve  L_II^T x_I = r_I       (diagonal block staged in LDS, one wavefront, lane per row)
//   update r_j -= sum_{i in I} L_ij x_i   for every j < 64 I
// Thread tid owns the stored positions p = tid + 1024 q of r (in registers), so the update
// reads the rows of block I coalesced with 64 independent loads per position.
constexpr int BSV_THREADS = 1024;

// BSV_Q: positions per thread (Np <= BSV_THREADS * BSV_Q)
template <int BSV_Q>
__global__ void __launch_bounds__(BSV_THREADS) backsolve_kernel(const double* __restrict__ Lall,
                                                                const double* __restrict__ vec,
                                                                int N, int Np, int64_t ld,
                                                                double* __restrict__ xl) {
    __shared__ double dg[64][65];
    __shared__ double rI[2][64];
    __shared__ double xI[2][64];
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    const double* Le = Lall + (size_t)e * (Np + 2) * ld;
    const double* s = vec + (size_t)e * 4 * N + 3 * N;
    double* xo = xl + (size_t)e * 2 * ld;
    double rx[BSV_Q], rl[BSV_Q];
#pragma unroll
    for (int q = 0; q < BSV_Q; ++q) {
        const int p = tid + BSV_THREADS * q;
        rx[q] = p < Np ? Le[(size_t)Np * ld + p] : 0.0;
        rl[q] = p < Np ? Le[(size_t)(Np + 1) * ld + p] : 0.0;
    }
    const int nJ = (Np + 63) / 64;
    for (int I = nJ - 1; I >= 0; --I) {
        const int c0 = 64 * I;
        const int wI = min(64, Np - c0);  // a multiple of 16
        for (int t = tid; t < 64 * 64; t += BSV_THREADS) {
            const int i = t >> 6, pp = t & 63;
            dg[i][pp] = (i < wI && pp < wI) ? Le[(size_t)(c0 + i) * ld + c0 + pp] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < BSV_Q; ++q) {
            const int p = tid + BSV_THREADS * q;
            if (p >= c0 && p < c0 + wI) {  // logical column perm16(p), row perm16(p) - c0
                const int m = perm16(p) - c0;
                rI[0][m] = rx[q];
                rI[1][m] = rl[q];
            }
        }
        __syncthreads();
        if (tid < 64) {
            const int m = tid;         // logical column c0 + m of the block
            const int pm = perm16(m);  // its stored position
            double ax = m < wI ? rI[0][m] : 0.0, al = m < wI ? rI[1][m] : 0.0;
            // lane m holds 1 / L_mm, so the sequential loop below only multiplies
            const double inv = m < wI ? 1.0 / dg[m][pm] : 0.0;
            for (int k = wI - 1; k >= 0; --k) {  // uniform loop, whole wavefront active
                const double ik = readlane_dbl(inv, k);
                const double xk = readlane_dbl(ax, k) * ik;
                const double lk = readlane_dbl(al, k) * ik;
                const double lkm = (m < k) ? dg[k][pm] : 0.0;
                ax = (m == k) ? xk : fma(-lkm, xk, ax);
                al = (m == k) ? lk : fma(-lkm, lk, al);
            }
            if (m < wI) {
                xI[0][m] = ax;
                xI[1][m] = al;
                if (c0 + m < N) {
                    xo[c0 + m] = s[c0 + m] * ax;
                    xo[ld + c0 + m] = s[c0 + m] * al;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < BSV_Q; ++q) {
            const int p = tid + BSV_THREADS * q;
            if (p < c0) {
                double ax = 0.0, al = 0.0;
                for (int i0 = 0; i0 < wI; i0 += 16) {  // 16 independent loads, then use
                    double lip[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i) lip[i] = Le[(size_t)(c0 + i0 + i) * ld + p];
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        ax = fma(lip[i], xI[0][i0 + i], ax);
                        al = fma(lip[i], xI[1][i0 + i], al);
                    }
                }
                rx[q] -= ax;
                rl[q] -= al;
            }
        }
        __syncthreads();  // dg, rI and xI are rewritten for the next block
    }
}

typedef __attribute__((address_space(3))) double lds_double;

// out = conj(M) in for a W x W complex block M (row-major, (re, im) pairs in LDS; the same
// address on every lane, so each read is a broadcast).
template <int W>
__device__ inline void conj_block_matvec(double2 (&out)[W], const double2 (&in)[W],
                                         const lds_double* M) {
#pragma unroll
    for (int y = 0; y < W; ++y) {
        double2 acc = cmk(0.0, 0.0);
#pragma unroll
        for (int x = 0; x < W; ++x)
            cfma(acc, cmk(M[2 * (y * W + x)], -M[2 * (y * W + x) + 1]), in[x]);
        out[y] = acc;
    }
}

// One thread per right-hand side c of one energy: c < N is column c of Q (d = v), c = N + b
// is column sp + b of R (d = u).  The forward sweep keeps y in Y[.][c]; the backward sweep
// overwrites it with q only where the assembly reads it (columns sq.. sq+W-1 and N..N+W-1),
// and for c < N accumulates, over the rows a of the column,
//   kd = sum_a G_ac u_a Q_ac,  kg = sum_a G_ac^2 u_a x_a,  pv = sum_a |G_ac|^2 v_a,  pu (u).
template <int W>
__global__ void __launch_bounds__(64) adjoint_solve_kernel(
    const double2* __restrict__ gL, const double2* __restrict__ Gc, const double* __restrict__ xl,
    const double* __restrict__ gamma, int L, double t, int64_t ld, int64_t ldY,
    uint32_t inject_lead, double2* __restrict__ Y, double2* __restrict__ part_k,
    double* __restrict__ part_p) {
    const int N = W * L;
    const int NC = N + W;
    const int e = blockIdx.y;
    // One wavefront per workgroup; the blocks gL_k are staged in LDS one slice ahead
    // (double-buffered, one barrier per slice); idle lanes compute on column 0.
    __shared__ double Ms_raw[2 * 2 * W * W];  // two buffers of W x W (re, im)
    const int tid = threadIdx.x;
    const int c = blockIdx.x * 64 + tid;
    const bool valid = c < NC;
    const bool dense = c < N;
    const int sp = inject_lead == 0 ? 0 : (L - 1) * W;
    const int sq = inject_lead == 0 ? (L - 1) * W : 0;
    const int col = dense ? c : (valid ? sp + (c - N) : 0);
    const bool keep_q = valid && (!dense || (c >= sq && c < sq + W));
    const int cl = valid ? c : 0;  // column that idle lanes read
    const double2* Ge = Gc + (size_t)e * N * ld;
    double2* Ye = Y + (size_t)e * N * ldY;
    const double* xe = xl + (size_t)e * 2 * ld;
    const double* le = xe + ld;
    const double2* gLe = gL + (size_t)e * L * W * W;
    lds_double* Ms = (lds_double*)Ms_raw;
    constexpr int BS = 2 * W * W;  // doubles per buffer
    // the 64 lanes copy block gL_slice into LDS buffer buf
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
        __syncthreads();  // block k visible in buffer k & 1; buffer (k + 1) & 1 no longer read
        const lds_double* cur = Ms + (k & 1) * BS;
        if (k + 1 < L) stage((k + 1) & 1, k + 1);
#pragma unroll
        for (int r = 0; r < W; ++r) {
            const int row = k * W + r;
            const double d = gamma[row] * (dense ? xe[row] : le[row]);
            const double2 g = Ge[(size_t)row * ld + col];
            z[r] = cmk(fma(d, g.x, -t * y[r].x), fma(d, g.y, -t * y[r].y));
        }
        conj_block_matvec<W>(y, z, cur);
        if (valid) {
#pragma unroll
            for (int r = 0; r < W; ++r) Ye[(size_t)(k * W + r) * ldY + c] = y[r];
        }
    }
    // y now holds y_{L-1} = q_{L-1}; the backward sweep stages gL_{L-2}, gL_{L-3}, ...
    double2 kd = cmk(0.0, 0.0), kg = cmk(0.0, 0.0);
    double pv = 0.0, pu = 0.0;
    __syncthreads();  // forward reads of both buffers done
    if (L > 1) stage(0, L - 2);
    for (int k = L - 1; k >= 0; --k) {
        if (k < L - 1) {
            const int j = L - 2 - k;  // 0, 1, ... : buffer parity
            __syncthreads();
            const lds_double* cur = Ms + (j & 1) * BS;
            if (k > 0) stage((j + 1) & 1, k - 1);
            conj_block_matvec<W>(z, y, cur);
#pragma unroll
            for (int r = 0; r < W; ++r) {
                const double2 yk = Ye[(size_t)(k * W + r) * ldY + cl];
                y[r] = cmk(fma(-t, z[r].x, yk.x), fma(-t, z[r].y, yk.y));
            }
        }
        if (keep_q) {
#pragma unroll
            for (int r = 0; r < W; ++r) Ye[(size_t)(k * W + r) * ldY + c] = y[r];
        }
        if (dense) {
#pragma unroll
            for (int r = 0; r < W; ++r) {
                const int row = k * W + r;
                const double2 g = Ge[(size_t)row * ld + col];
                const double gm = gamma[row];
                const double ua = gm * le[row], va = gm * xe[row];
                cfma(kd, cscale(g, ua), y[r]);
                kg = cadd(kg, cscale(cmul(g, g), ua * xe[row]));
                const double p = cabs2(g);
                pv = fma(p, va, pv);
                pu = fma(p, ua, pu);
            }
        }
    }
    if (dense) {
        part_k[((size_t)e * 2 + 0) * N + c] = kd;
        part_k[((size_t)e * 2 + 1) * N + c] = kg;
        part_p[((size_t)e * 2 + 0) * N + c] = pv;
        part_p[((size_t)e * 2 + 1) * N + c] = pu;
    }
}

// Per energy and site i: K_i and the explicit gamma terms (see the top of the file), from
// the column partials of adjoint_solve_kernel, the rows i of Q (columns sq..) and R
// (columns N..) in Y, and the slice entries G_{sp+c,i}, G_{sq+c,i}.
template <int W>
__global__ void __launch_bounds__(256) grad_assemble_kernel(
    const double2* __restrict__ Gc, const double2* __restrict__ Y, const double* __restrict__ xl,
    const double* __restrict__ gamma, const double* __restrict__ wL, const double* __restrict__ wR,
    const double* __restrict__ Adiag, const double* __restrict__ gam_lead,
    const double2* __restrict__ corner, const double2* __restrict__ part_k,
    const double* __restrict__ part_p, int L, int64_t ld, int64_t ldY, uint32_t inject_lead,
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
    const double2* Yi = Y + ((size_t)e * N + i) * ldY;
    const double* xe = xl + (size_t)e * 2 * ld;
    const double* le = xe + ld;
    const double2 kd = part_k[((size_t)e * 2 + 0) * N + i];
    const double2 kg = part_k[((size_t)e * 2 + 1) * N + i];
    const double pv = part_p[((size_t)e * 2 + 0) * N + i];
    const double pu = part_p[((size_t)e * 2 + 1) * N + i];
    double2 K = cadd(cscale(kd, 2.0), cmk(2.0 * kg.y, -2.0 * kg.x));  // 2 kd - 2i kg
    // lead terms: 2 sum_b al_b (Gamma_p G_{p,i})_b + 2 sum_b be_b (Gamma_q G_{q,i})_b with
    // al_b = conj(R_{i,sp+b}), be_b = conj(Q_{i,sq+b})
    double2 gpi[W], gqi[W];
#pragma unroll
    for (int c = 0; c < W; ++c) {
        gpi[c] = Ge[(size_t)(sp + c) * ld + i];
        gqi[c] = Ge[(size_t)(sq + c) * ld + i];
    }
#pragma unroll 1
    for (int b = 0; b < W; ++b) {
        double2 tp = cmk(0.0, 0.0), tq = cmk(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < W; ++c) {
            tp = cadd(tp, cscale(gpi[c], gm[b * W + c]));
            tq = cadd(tq, cscale(gqi[c], gm[b * W + c]));
        }
        const double2 al = cconj(Yi[N + b]);
        const double2 be = cconj(Yi[sq + b]);
        K = cadd(K, cscale(cadd(cmul(al, tp), cmul(be, tq)), 2.0));
    }
    // T_qp term: sum_{a in q, b in p} G_ia Psi5_ab G_bi
#pragma unroll 1
    for (int a = 0; a < W; ++a) {
        double2 s = cmk(0.0, 0.0);
#pragma unroll
        for (int b = 0; b < W; ++b) s = cadd(s, cmul(psi5[a * W + b], gpi[b]));
        K = cadd(K, cmul(Ge[(size_t)(sq + a) * ld + i], s));
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

template <int W>
static hipError_t launch_adjoint_w(const mcnegf_kernel& k, const GradBuffers& gb,
                                   uint32_t inject_lead, hipStream_t s) {
    {
        MCNEGF_TIMED("adjoint_solve_kernel", s);
        hipLaunchKernelGGL(adjoint_solve_kernel<W>, dim3((k.N + W + 63) / 64, k.nE), dim3(64),
                           0, s, reinterpret_cast<const double2*>(k.gL), gb.G, gb.xl, k.gamma, k.L,
                           k.t, gb.ld, gb.ldY, inject_lead, gb.Y, gb.part_k, gb.part_p);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    {
        MCNEGF_TIMED("grad_assemble_kernel", s);
        hipLaunchKernelGGL(grad_assemble_kernel<W>, dim3((k.N + 255) / 256, k.nE), dim3(256), 0,
                           s, gb.G, gb.Y, gb.xl, k.gamma, k.wL, k.wR, k.Adiag, k.gam_lead,
                           reinterpret_cast<const double2*>(k.corner), gb.part_k, gb.part_p, k.L,
                           gb.ld, gb.ldY, inject_lead, gb.gV, gb.gG);
    }
    return hipGetLastError();
}

static hipError_t launch_backsolve(const mcnegf_kernel& k, double* xl, hipStream_t s) {
    const int N = k.N, nE = k.nE;
    const int Np = (int)k.p_pitch;
    {
        MCNEGF_TIMED("backsolve_kernel", s);
        if (Np <= BSV_THREADS * 4)
            hipLaunchKernelGGL(backsolve_kernel<4>, dim3(nE), dim3(BSV_THREADS), 0, s, k.direct,
                               k.direct_vec, N, Np, k.p_pitch, xl);
        else if (Np <= BSV_THREADS * 8)
            hipLaunchKernelGGL(backsolve_kernel<8>, dim3(nE), dim3(BSV_THREADS), 0, s, k.direct,
                               k.direct_vec, N, Np, k.p_pitch, xl);
        else
            hipLaunchKernelGGL(backsolve_kernel<16>, dim3(nE), dim3(BSV_THREADS), 0, s, k.direct,
                               k.direct_vec, N, Np, k.p_pitch, xl);
    }
    return hipGetLastError();
}

// Energies are processed in chunks of `chunk`: the complex G, the adjoint solves and the
// per-site partials of one chunk live in the workspace at a time (the stored RGF blocks of
// every energy regenerate each chunk's G); gV, gG hold every energy for the final sum.
hipError_t launch_grad(const mcnegf_kernel& k, const GradBuffers& gb, uint32_t inject_lead,
                       const double* weights, double* dI_dV, double* dI_dgamma, int chunk,
                       hipStream_t s) {
    const int N = k.N, nE = k.nE;
    hipError_t err;
    for (int e0 = 0; e0 < nE; e0 += chunk) {
        const int nc = min(chunk, nE - e0);
        const mcnegf_kernel kc = energy_slice(k, e0, nc);
        GradBuffers g = gb;
        g.gV = gb.gV + (size_t)e0 * N;
        g.gG = gb.gG + (size_t)e0 * N;
        if ((err = launch_backsolve(kc, g.xl, s)) != hipSuccess) return err;
        if ((err = launch_fullinv_store_g(kc, g.G, g.ld, s)) != hipSuccess) return err;
        switch (k.W) {
#define MCNEGF_CASE(w)                                                         \
    case w:                                                                    \
        if ((err = launch_adjoint_w<w>(kc, g, inject_lead, s)) != hipSuccess) \
            return err;                                                        \
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

hipError_t launch_grad_reduce(const GradBuffers& gb, const double* weights, int nE, int N,
                              double* dI_dV, double* dI_dgamma, hipStream_t s) {
    {
        MCNEGF_TIMED("grad_reduce_kernel", s);
        hipLaunchKernelGGL(grad_reduce_kernel, dim3((N + 255) / 256), dim3(256), 0, s, gb.gV,
                           gb.gG, weights, nE, N, dI_dV, dI_dgamma);
    }
    return hipGetLastError();
}

}  // namespace mcnegf
