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
// in the symmetrically scaled form S M S = L L^T with S = diag(M_jj^{-1/2}); probes with
// gamma_j = 0 decouple (identity row).  Then
//   T_k = T_qp + sum_j T_qj n_j = T_qp + (L^{-1} S T_q) . (L^{-1} S T_p),
// so only forward substitutions are needed; they come out of the factorization itself when
// the two vectors (S T_p)^T and (S T_q)^T are appended below the matrix as two extra rows.
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

// Energy-resolved current of inelastic walks (step 7'): a walker injected at lead p at energy
// e0 scores c_p(e0) at its exit, so the exits at lead r with energy e give
//   S[r][e] = sum_e0 w_e0 c_p(e0) hist[r][e0][e] / N_e0
// (N_e0 the walkers injected at e0, truncated ones included); sum_e S[q][e] is the current of
// the tallies.  One thread per (r, e); the sum over e0 runs in order.
__global__ void __launch_bounds__(256) spectrum_kernel(const int64_t* __restrict__ tallies,
                                                       const int64_t* __restrict__ hist,
                                                       const double* __restrict__ lead,
                                                       const double* __restrict__ weights,
                                                       int nE, uint32_t inject_lead,
                                                       double* __restrict__ S) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * nE) return;
    const int r = idx / nE, e = idx % nE;
    double acc = 0.0;
    for (int e0 = 0; e0 < nE; ++e0) {
        const int64_t* t = tallies + (size_t)e0 * MCNEGF_TALLY_N;
        const int64_t nw = t[MCNEGF_TALLY_EXIT_L] + t[MCNEGF_TALLY_EXIT_R] + t[MCNEGF_TALLY_TRUNC];
        const int64_t h = hist[((size_t)r * nE + e0) * nE + e];
        if (nw <= 0 || h == 0) continue;
        const double c = lead[(size_t)e0 * MCNEGF_LEAD_NTERMS +
                              (inject_lead == 0 ? MCNEGF_LEAD_CL : MCNEGF_LEAD_CR)];
        acc += weights[e0] * c / (double)nw * (double)h;
    }
    S[idx] = acc;
}

hipError_t launch_spectrum(const mcnegf_kernel& k, uint32_t inject_lead, const int64_t* tallies,
                           const int64_t* hist, const double* weights, double* spectrum,
                           hipStream_t s) {
    {
        MCNEGF_TIMED("spectrum_kernel", s);
        hipLaunchKernelGGL(spectrum_kernel, dim3((2 * k.nE + 255) / 256), dim3(256), 0, s,
                           tallies, hist, k.lead, weights, k.nE, inject_lead, spectrum);
    }
    return hipGetLastError();
}

// Importance-sampled walks (Sec. V A, "Improved estimator"): per energy the N_k walkers'
// scores (path likelihood ratios at an exit at q, else 0) have sums S1, S2; then
//   T_k = c_p S1 / N_k,  sigma_k = c_p sqrt(s^2 / N_k),  s^2 = (S2 - S1^2 / N_k) / (N_k - 1).
__global__ void weighted_current_kernel(const int64_t* __restrict__ tallies,
                                        const double* __restrict__ wsum,
                                        const double* __restrict__ lead, int nE,
                                        uint32_t inject_lead, double* __restrict__ T,
                                        double* __restrict__ sig) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nE) return;
    const int64_t* t = tallies + (size_t)k * MCNEGF_TALLY_N;
    const double walkers =
        (double)(t[MCNEGF_TALLY_EXIT_L] + t[MCNEGF_TALLY_EXIT_R] + t[MCNEGF_TALLY_TRUNC]);
    const double c = lead[(size_t)k * MCNEGF_LEAD_NTERMS +
                          (inject_lead == 0 ? MCNEGF_LEAD_CL : MCNEGF_LEAD_CR)];
    if (walkers <= 0.0) {
        T[k] = 0.0;
        sig[k] = 0.0;
        return;
    }
    const double s1 = wsum[2 * (size_t)k], s2 = wsum[2 * (size_t)k + 1];
    T[k] = c * s1 / walkers;
    const double var = walkers > 1.0 ? fmax(s2 - s1 * s1 / walkers, 0.0) / (walkers - 1.0) : 0.0;
    sig[k] = c * sqrt(var / walkers);
}

hipError_t launch_weighted_current(const mcnegf_kernel& k, uint32_t inject_lead,
                                   const int64_t* tallies, const double* wsum,
                                   const double* weights, double* T, double* sigmaT,
                                   hipStream_t s) {
    {
        MCNEGF_TIMED("weighted_current_kernel", s);
        hipLaunchKernelGGL(weighted_current_kernel, dim3((k.nE + 255) / 256), dim3(256), 0, s,
                           tallies, wsum, k.lead, k.nE, inject_lead, T, sigmaT);
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

// Interpolated walks (Sec. V A, "Interpolation"): fine energy f between the built energies
// E_lo and E_hi with mixture weight alpha = a32 / 2^32 (the one its walks used); the row total
// that scales the estimator is interpolated like the rows, c = (1 - alpha) c_lo + alpha c_hi,
// then T_f and sigma_f as in MC mode.
__global__ void interp_current_kernel(const int64_t* __restrict__ tallies,
                                      const double* __restrict__ lead,
                                      const double* __restrict__ nodes, uint32_t nE,
                                      const double* __restrict__ fine, int nF,
                                      uint32_t inject_lead, double* __restrict__ T,
                                      double* __restrict__ sig, uint32_t* __restrict__ status) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nF) return;
    uint32_t lo, a32;
    bool bad;
    interp_bracket(nodes, nE, fine[f], lo, a32, bad);
    if (bad) atomicOr(status, MCNEGF_FLAG_RANGE);
    const uint32_t hi = lo + 1 < nE ? lo + 1 : lo;
    const int slot = inject_lead == 0 ? MCNEGF_LEAD_CL : MCNEGF_LEAD_CR;
    const double alpha = (double)a32 * 0x1.0p-32;
    const double c = (1.0 - alpha) * lead[(size_t)lo * MCNEGF_LEAD_NTERMS + slot] +
                     alpha * lead[(size_t)hi * MCNEGF_LEAD_NTERMS + slot];
    const int64_t* t = tallies + (size_t)f * MCNEGF_TALLY_N;
    const double walkers =
        (double)(t[MCNEGF_TALLY_EXIT_L] + t[MCNEGF_TALLY_EXIT_R] + t[MCNEGF_TALLY_TRUNC]);
    const double hits = (double)(inject_lead == 0 ? t[MCNEGF_TALLY_EXIT_R] : t[MCNEGF_TALLY_EXIT_L]);
    if (walkers <= 0.0) {
        T[f] = 0.0;
        sig[f] = 0.0;
        return;
    }
    const double p = hits / walkers;
    T[f] = c * p;
    sig[f] = walkers > 1.0 ? c * sqrt(p * (1.0 - p) / (walkers - 1.0)) : 0.0;
}

hipError_t launch_interp_current(const mcnegf_kernel& k, const double* fine, uint32_t nF,
                                 uint32_t inject_lead, const int64_t* tallies,
                                 const double* weights, double* T, double* sigmaT,
                                 hipStream_t s) {
    {
        MCNEGF_TIMED("interp_current_kernel", s);
        hipLaunchKernelGGL(interp_current_kernel, dim3((nF + 255) / 256), dim3(256), 0, s,
                           tallies, k.lead, k.energies, (uint32_t)k.nE, fine, (int)nF,
                           inject_lead, T, sigmaT, k.status);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    {
        MCNEGF_TIMED("current_sum_kernel", s);
        hipLaunchKernelGGL(current_sum_kernel, dim3(1), dim3(256), 0, s, T, sigmaT, weights,
                           (int)nF, k.reduce);
    }
    return hipGetLastError();
}

// Energies drawn with probability w_k / W (W = sum_k w_k, Sec. II F step 2 with h = w / W)
// and the estimator of the linear-response transmission with h proportional to the weight
// (Sec. II G, Eq. (66) read with f -> w): X = W c_p(E_k) for an exit at q, else 0, so that
// E[X] = sum_k w_k T_k.  Over the N walkers of the tallies: I = W S1 / N with
// S1 = sum_k c_k R_k (R_k exits at q), and sigma_I^2 = (W^2 S2 / N - I^2) / (N - 1) with
// S2 = sum_k c_k^2 R_k (the sample variance of X over N).  T_k and sigma_k are the per-energy
// ratios as in MC mode.  out[0] = I, out[1] = sigma_I^2.
__global__ void __launch_bounds__(256) sampled_current_kernel(const int64_t* __restrict__ tallies,
                                                              const double* __restrict__ lead,
                                                              const double* __restrict__ w,
                                                              int nE, uint32_t inject_lead,
                                                              double* __restrict__ T,
                                                              double* __restrict__ sig,
                                                              double* __restrict__ out) {
    __shared__ double red[256];
    double sw = 0.0, s1 = 0.0, s2 = 0.0, nw = 0.0;
    for (int k = threadIdx.x; k < nE; k += 256) {
        const int64_t* t = tallies + (size_t)k * MCNEGF_TALLY_N;
        const double walkers =
            (double)(t[MCNEGF_TALLY_EXIT_L] + t[MCNEGF_TALLY_EXIT_R] + t[MCNEGF_TALLY_TRUNC]);
        const double hits =
            (double)(inject_lead == 0 ? t[MCNEGF_TALLY_EXIT_R] : t[MCNEGF_TALLY_EXIT_L]);
        const double c = lead[(size_t)k * MCNEGF_LEAD_NTERMS +
                              (inject_lead == 0 ? MCNEGF_LEAD_CL : MCNEGF_LEAD_CR)];
        sw += w[k];
        s1 += c * hits;
        s2 += c * c * hits;
        nw += walkers;
        const double p = walkers > 0.0 ? hits / walkers : 0.0;
        T[k] = c * p;
        sig[k] = walkers > 1.0 ? c * sqrt(p * (1.0 - p) / (walkers - 1.0)) : 0.0;
    }
    sw = block_reduce256(sw, red);
    s1 = block_reduce256(s1, red);
    s2 = block_reduce256(s2, red);
    nw = block_reduce256(nw, red);
    if (threadIdx.x == 0) {
        const double I = nw > 0.0 ? sw * s1 / nw : 0.0;
        const double m2 = nw > 0.0 ? sw * sw * s2 / nw : 0.0;
        const double var = nw > 1.0 ? (m2 - I * I) / (nw - 1.0) : 0.0;
        out[0] = I;
        out[1] = var > 0.0 ? var : 0.0;
    }
}

hipError_t launch_sampled_current(const mcnegf_kernel& k, uint32_t inject_lead,
                                  const int64_t* tallies, const double* weights, double* T,
                                  double* sigmaT, hipStream_t s) {
    {
        MCNEGF_TIMED("sampled_current_kernel", s);
        hipLaunchKernelGGL(sampled_current_kernel, dim3(1), dim3(256), 0, s, tallies, k.lead,
                           weights, k.nE, inject_lead, T, sigmaT, k.reduce);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- DIRECT
// vec layout per energy: [0] u_j = gamma_j s_j, [1] u_j w_p(j), [2] u_j w_q(j), [3] s_j,
// with s_j = M_jj^{-1/2} (0 for a decoupled probe) and w_p, w_q the exit weights of the
// injecting and the collecting lead.  Scaled matrix: 1 on the diagonal, -u_i u_j |G_ij|^2 off it;
// scaled right-hand sides: u_j w_p(j) and u_j w_q(j).
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
    const double u = g * sj;
    double* v = vec + (size_t)e * 4 * N;
    v[j] = u;
    v[N + j] = u * wp;
    v[2 * N + j] = u * wq;
    v[3 * N + j] = sj;
}

// ---- Left-looking blocked Cholesky of the bordered probe system on FP64 matrix cores.
//
// Per energy, logical rows 0..Np-1 are the scaled matrix padded with identity rows up to
// Np = round_up(N, 16), rows Np and Np+1 are the two scaled right-hand sides; columns
// 0..Np-1 are factored.  Block column J (columns c0 = 64 J .. c0 + wJ - 1):
//   V  = A[c0:, J] - L[c0:, 0:c0] L[J, 0:c0]^T      (update, MFMA)
//   L_JJ = chol(V_JJ),  Z = L_JJ^{-1}                (one wavefront, lane per row / column)
//   L[below, J] = V_below L_JJ^{-T}   computed as (Z V_below^T)^T   (MFMA)
// After the last block column, rows Np and Np+1 of L hold L^{-1} S T_p and L^{-1} S T_q.
// One workgroup of 8 wavefronts per energy; each wavefront owns two 16-row tiles (w, w + 8) of a
// 256-row super-tile and keeps their 16 x 64 updates in accumulators.  Block-column rows
// L[J, 0:c0] are staged through LDS in 64-wide K chunks and serve as the MFMA A operand;
// the tile rows stream from global memory as the B operand, so the accumulator holds the
// transposed update, which is directly the B operand of the triangular-solve product.
// v_mfma_f64_16x16x4f64 operand layouts (lane l, g = l / 16, n = l % 16):
//   A[m][k]: m = n, k = g;   B[k][c]: k = g, c = n;   D[i][c] (item r): i = 4 r + g, c = n.
// A lane's four accumulator items are therefore the columns 4 r + g of a 16-column block.
// Rows of L are stored with the columns of every 16-column block permuted so that these
// four items are contiguous (logical column 4 r + g at position 4 g + r, an involution):
// the update contracts over stored positions of two rows of L, which any common column
// permutation leaves unchanged, and the two bordered rows enter only through their dot
// product, which it leaves unchanged too.
typedef double dmfma4 __attribute__((ext_vector_type(4)));

constexpr int CH_NB = 64;            // block-column width
constexpr int CH_KC = 32;            // K chunk staged in LDS (double-buffered)
constexpr int CH_BP = CH_KC + 4;     // LDS pitch of a staged row (doubles)
constexpr int CH_KG = CH_KC / 16;    // 16-column MFMA groups per chunk
constexpr int CH_VP = CH_NB + 1;     // LDS pitch of the diagonal block
constexpr int CH_WAVES = 8;
constexpr int CH_ROWS = CH_WAVES * 32;  // rows per super-tile

struct CholArgs {
    const double* P;      // [nE][N][ld] |G_ij|^2
    const double* vec;    // [nE][4][N]
    const double* lead;   // [nE][8]
    double* Lall;         // [nE][Np + 2][ld]
    double* T;
    double* sig;
    uint32_t* status;
    int N, Np;
    int64_t ld;
    uint32_t inject_lead;
    // Block columns [J0, J1) in this launch, and workgroups per energy.  One launch over all
    // block columns (nsplit = 1) also forms T from the bordered rows as it goes; with several
    // launches (one per block column, nsplit workgroups per energy taking every nsplit-th
    // super-tile) T is formed afterwards by direct_dot_kernel.
    int J0, J1, nsplit;
    bool single;
};

__device__ inline double readlane_f64(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Entries (i, c + 4 r), r = 0..3, of the bordered scaled matrix (lower part, c + 12 < Np).
__device__ inline void aorig4(const CholArgs& a, const double* Pe, const double* ve, int i, int c,
                              double (&out)[4]) {
    const int N = a.N;
    if (i < N) {
        const double* Pr = Pe + (size_t)i * a.ld;
        const double ui = ve[i];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = c + 4 * r;
            const double uj = j < N ? ve[j] : 0.0;
            const double pij = Pr[j];
            out[r] = (j == i) ? 1.0 : (j < N ? -ui * uj * pij : 0.0);
        }
    } else if (i < a.Np) {
#pragma unroll
        for (int r = 0; r < 4; ++r) out[r] = (c + 4 * r == i) ? 1.0 : 0.0;
    } else if (i < a.Np + 2) {
        const double* rhs = ve + (size_t)(i - a.Np + 1) * N;
#pragma unroll
        for (int r = 0; r < 4; ++r) out[r] = (c + 4 * r < N) ? rhs[c + 4 * r] : 0.0;
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) out[r] = 0.0;
    }
}

// Staging of a block-column row segment (4 doubles at column col) through registers into LDS.
// Rows beyond R read row R - 1 and are then scaled by 0 (a select would let the compiler turn
// the load into a predicated one, and the branch around it makes every later wait for any load
// a wait for all of them, the prefetched tile rows included).  Such rows only feed results
// that are never stored (rows or columns beyond the matrix), so a non-finite value there is
// harmless.
__device__ inline double4 stage_load(const double* Le, int64_t ld, int R, int row, int col) {
    const bool ok = row < R;
    const double4 v = *reinterpret_cast<const double4*>(Le + (size_t)(ok ? row : R - 1) * ld + col);
    const double m = ok ? 1.0 : 0.0;
    return double4{v.x * m, v.y * m, v.z * m, v.w * m};
}

// MFMAs of one staged chunk for the first NT of a wavefront's two 16-row tiles: NCB 16-column
// blocks of the block column (A operand from LDS), tile rows (B operand) from registers.
template <int NCB, int NT = 2>
__device__ inline void chunk_mfma(const double* B, const double4 (&av)[2][CH_KG],
                                  dmfma4 (&acc)[2][4], int ln, int cq) {
#pragma unroll
    for (int kg = 0; kg < CH_KG; ++kg) {
        double4 bf[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
            bf[cb] = *reinterpret_cast<const double4*>(&B[(16 * cb + ln) * CH_BP + 16 * kg + cq]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double bv = q == 0 ? av[t][kg].x : q == 1 ? av[t][kg].y
                                : q == 2 ? av[t][kg].z : av[t][kg].w;
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    const double aval = q == 0 ? bf[cb].x : q == 1 ? bf[cb].y
                                      : q == 2 ? bf[cb].z : bf[cb].w;
                    acc[t][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aval, bv, acc[t][cb], 0, 0, 0);
                }
            }
        }
    }
}

__device__ inline void stage_store(double* Bs, int sm, int sc, const double4& b) {
    *reinterpret_cast<double4*>(&Bs[sm * CH_BP + sc]) = b;
}

// The LDS arguments carry the LDS address space so that every access is a DS instruction: the
// lanes exchange rows and columns through LDS, which a wavefront's DS instructions see in
// program order (generic pointers would turn them into FLAT accesses, which give no such order).
typedef __attribute__((address_space(3))) double lds_double;
typedef __attribute__((address_space(3))) int lds_int;

__device__ __noinline__ void factor_diag_block(lds_double* VZs, lds_double* Ls, lds_double* colbuf,
                                               double* Lg, int64_t ld, int wJ, int lane,
                                               lds_int* bad_flag, bool store) {
    // Lane i holds row i; column k is shared through LDS.  The step branch is uniform; the
    // updates of columns from wJ on are harmless (their entries stay zero).
    const int i = lane;
    double rw[CH_NB];
#pragma unroll
    for (int j = 0; j < CH_NB; ++j) rw[j] = (i < wJ && j < wJ && j <= i) ? VZs[i * CH_VP + j] : 0.0;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < CH_NB; ++k) {
        if (k < wJ) {
            double piv = readlane_f64(rw[k], k);
            const bool good = piv > 0.0 && isfinite(piv);
            bad |= !good;
            piv = good ? piv : 1.0;
            // one reciprocal square root and a product per lane: a shorter dependent chain
            // per pivot than a square root followed by a division
            const double rs = rsqrt(piv);
            const double lik = (i >= k) ? rw[k] * rs : 0.0;
            rw[k] = lik;
            colbuf[i] = lik;
#pragma unroll
            for (int j = k + 1; j < CH_NB; ++j) {
                rw[j] = fma(-lik, colbuf[j], rw[j]);
            }
        }
    }
    if (bad && lane == 0) *bad_flag = 1;
#pragma unroll
    for (int j = 0; j < CH_NB; ++j) {
        const double lv = (j <= i && i < wJ) ? rw[j] : (i == j ? 1.0 : 0.0);
        Ls[i * CH_VP + j] = lv;
        if (store && j <= i && i < wJ)
            Lg[(size_t)i * ld + (j & ~15) + 4 * (j & 3) + ((j >> 2) & 3)] = lv;
    }
    // Inverses of the four 16 x 16 diagonal sub-blocks of L_JJ: lane (b, c) = (lane / 16,
    // lane % 16) computes column c of L_bb^{-1} by forward substitution and stores it in the
    // diagonal sub-block b of V (Ls was written by this wavefront, whose LDS accesses stay in
    // order).
    const int b = lane >> 4, c = lane & 15;
    const lds_double* Lb = Ls + (16 * b) * CH_VP + 16 * b;
    double z[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        double s0 = (r == c) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
        for (int m = 0; m + 1 < r; m += 2) {
            s0 = fma(-Lb[r * CH_VP + m], z[m], s0);
            s1 = fma(-Lb[r * CH_VP + m + 1], z[m + 1], s1);
        }
        if (r & 1) s0 = fma(-Lb[r * CH_VP + r - 1], z[r - 1], s0);
        z[r] = (s0 + s1) / Lb[r * CH_VP + r];
    }
    lds_double* Zb = VZs + (16 * b) * CH_VP + 16 * b;
#pragma unroll
    for (int r = 0; r < 16; ++r) Zb[r * CH_VP + c] = z[r];
}

__global__ void __launch_bounds__(512) cholesky_kernel(CholArgs a) {
    __shared__ double Bs[2][CH_NB * CH_BP];  // double-buffered K chunk of block-column rows
    __shared__ double VZs[CH_NB * CH_VP];  // diagonal block V, then Z = L_JJ^{-1}
    __shared__ double Ls[CH_NB * CH_VP];   // L_JJ
    __shared__ double colbuf[CH_NB];
    __shared__ double dot_acc;
    __shared__ int bad_flag;

    const int e = blockIdx.x / a.nsplit;
    const int part = blockIdx.x - e * a.nsplit;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ln = lane & 15;
    const int g = lane >> 4;
    const int cq = 4 * g;
    const int Np = a.Np;
    const int R = Np + 2;
    const int64_t ld = a.ld;
    const double* Pe = a.P + (size_t)e * a.N * ld;
    const double* ve = a.vec + (size_t)e * 4 * a.N;
    double* Le = a.Lall + (size_t)e * R * ld;
    if (tid == 0) {
        dot_acc = 0.0;
        bad_flag = 0;
    }
    // staging assignment: row sm of the block column, 4 doubles at column sc of a chunk
    const int sm = tid >> 3;
    const int sc = (tid & 7) * 4;

    for (int J = a.J0; J < a.J1; ++J) {
        const int c0 = J * CH_NB;
        const int wJ = min(CH_NB, Np - c0);
        const int ncb = wJ >> 4;
        // rows of L written below the previous diagonal block (by any wavefront) are read next
        __syncthreads();

        // ---- diagonal block: V_JJ = A_JJ - L[J, 0:c0] L[J, 0:c0]^T, both operands from LDS.
        // Wavefront w owns the 16 x 16 blocks p = w and p = w + 8 (block row p / 4, column p % 4).
        {
            dmfma4 accd[2] = {dmfma4{0.0, 0.0, 0.0, 0.0}, dmfma4{0.0, 0.0, 0.0, 0.0}};
            // chunk it + 1 is in registers while chunk it + 2 is loaded (two chunks ahead: this
            // pass has little MFMA work to cover a load); loads past the last chunk re-read it
            // and their data is never used, so neither loads nor stores are predicated
            double4 bnext = {0.0, 0.0, 0.0, 0.0};
            if (c0 > 0) {
                stage_store(Bs[0], sm, sc, stage_load(Le, ld, R, c0 + sm, sc));
                bnext = stage_load(Le, ld, R, c0 + sm, min(CH_KC, c0 - CH_KC) + sc);
                __syncthreads();
            }
            for (int kc = 0, it = 0; kc < c0; kc += CH_KC, ++it) {
                const double* B = Bs[it & 1];
                const double4 bst = bnext;
                bnext = stage_load(Le, ld, R, c0 + sm, min(kc + 2 * CH_KC, c0 - CH_KC) + sc);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int p = wave + 8 * h;
                    const int tb = p >> 2, cb = p & 3;
                    if (cb <= tb && tb < ncb) {
#pragma unroll
                        for (int kg = 0; kg < CH_KG; ++kg) {
                            const double4 av = *reinterpret_cast<const double4*>(
                                &B[(16 * cb + ln) * CH_BP + 16 * kg + cq]);
                            const double4 bv = *reinterpret_cast<const double4*>(
                                &B[(16 * tb + ln) * CH_BP + 16 * kg + cq]);
                            accd[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, accd[h], 0, 0, 0);
                            accd[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.y, accd[h], 0, 0, 0);
                            accd[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.z, bv.z, accd[h], 0, 0, 0);
                            accd[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.w, bv.w, accd[h], 0, 0, 0);
                        }
                    }
                }
                stage_store(Bs[(it & 1) ^ 1], sm, sc, bst);  // unread after the last chunk
                __syncthreads();
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int p = wave + 8 * h;
                const int tb = p >> 2, cb = p & 3;
                if (cb <= tb && tb < ncb) {
                    double ao[4];
                    aorig4(a, Pe, ve, c0 + 16 * tb + ln, c0 + 16 * cb + g, ao);
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        VZs[(16 * tb + ln) * CH_VP + 16 * cb + 4 * r + g] = ao[r] - accd[h][r];
                }
            }
        }
        __syncthreads();
        if (wave == 0)
            factor_diag_block((lds_double*)VZs, (lds_double*)Ls, (lds_double*)colbuf,
                              Le + (size_t)c0 * ld + c0, ld, wJ, lane, (lds_int*)&bad_flag,
                              part == 0);
        __syncthreads();

        // ---- rows below the diagonal block, in super-tiles of 256 rows
        for (int st = c0 + wJ + part * CH_ROWS; st < R; st += a.nsplit * CH_ROWS) {
            // this wave's tiles: rows rw[t] .. rw[t] + 15 for t = 0, 1, tile wave + 8 t of the
            // super-tile, so that a partial super-tile gives each wavefront at most one tile
            // when it holds at most 8 (the wavefronts' MFMA work is then halved)
            const int rw[2] = {st + 16 * wave, st + 16 * (wave + 8)};
            dmfma4 acc[2][4];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) acc[t][cb] = dmfma4{0.0, 0.0, 0.0, 0.0};

            // update: acc^T = L[tile rows, 0:c0] . L[J rows, 0:c0]^T.  Chunk it of the
            // block-column rows is in Bs[it & 1] while chunk it + 1 is staged into the other
            // buffer and this wavefront's tile rows of chunk it + 1 are loaded: one barrier per
            // chunk, loads in flight across the chunk's MFMAs.
            if (c0 > 0) {
                double4 av[2][CH_KG];
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int kg = 0; kg < CH_KG; ++kg)
                        av[t][kg] = stage_load(Le, ld, R, rw[t] + ln, 16 * kg + cq);
                stage_store(Bs[0], sm, sc, stage_load(Le, ld, R, c0 + sm, sc));
                __syncthreads();
                // c0 = 64 J is a whole number of chunk pairs: the loop takes two chunks per
                // iteration in straight-line code, the tile rows alternating between two
                // register sets (chunk 2i multiplies av while an is loaded, chunk 2i + 1 the
                // reverse) and the staged block-column rows between the two LDS buffers, so
                // neither the loads nor the accumulators are copied.  All four 16-column
                // blocks are multiplied (a narrower last block column's extra blocks are
                // never stored), so the accumulators keep their registers.
                double4 an[2][CH_KG];
                for (int kc = 0; kc < c0; kc += 2 * CH_KC) {
                    {
                        const int kn = kc + CH_KC;  // always inside: c0 is a multiple of 64
                        const double4 bst = stage_load(Le, ld, R, c0 + sm, kn + sc);
#pragma unroll
                        for (int t = 0; t < 2; ++t)
#pragma unroll
                            for (int kg = 0; kg < CH_KG; ++kg)
                                an[t][kg] = stage_load(Le, ld, R, rw[t] + ln, kn + 16 * kg + cq);
                        if (rw[1] < R) chunk_mfma<4, 2>(Bs[0], av, acc, ln, cq);
                        else if (rw[0] < R) chunk_mfma<4, 1>(Bs[0], av, acc, ln, cq);
                        stage_store(Bs[1], sm, sc, bst);
                        __syncthreads();
                    }
                    {
                        const bool more = kc + 2 * CH_KC < c0;
                        const int kn = more ? kc + 2 * CH_KC : kc + CH_KC;
                        const double4 bst = stage_load(Le, ld, R, c0 + sm, kn + sc);
#pragma unroll
                        for (int t = 0; t < 2; ++t)
#pragma unroll
                            for (int kg = 0; kg < CH_KG; ++kg)
                                av[t][kg] = stage_load(Le, ld, R, rw[t] + ln, kn + 16 * kg + cq);
                        if (rw[1] < R) chunk_mfma<4, 2>(Bs[1], an, acc, ln, cq);
                        else if (rw[0] < R) chunk_mfma<4, 1>(Bs[1], an, acc, ln, cq);
                        if (more) stage_store(Bs[0], sm, sc, bst);
                        __syncthreads();
                    }
                }
            }
            // V = A - update (lane: row rw[t] + ln, columns c0 + 16 cb + 4 r + g), then
            // X L_JJ^T = V by 16-column blocks: X_b^T = L_bb^{-1} (V_b^T - sum_{a<b} L_ba X_a^T),
            // stored as rows of L.  V^T and X^T blocks are in accumulator layout, which is the
            // B-operand layout of the next product.
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int rt = rw[t];
                if (rt < R) {
                    dmfma4 y[4];
#pragma unroll
                    for (int cb = 0; cb < 4; ++cb) {
                        double ao[4];
                        if (cb < ncb) aorig4(a, Pe, ve, rt + ln, c0 + 16 * cb + g, ao);
                        else ao[0] = ao[1] = ao[2] = ao[3] = 0.0;
                        // blocks beyond the block column's width hold the unused products of
                        // the update: zero, as the bordered rows' dot product below reads them
#pragma unroll
                        for (int r = 0; r < 4; ++r) y[cb][r] = cb < ncb ? ao[r] - acc[t][cb][r] : 0.0;
                    }
#pragma unroll
                    for (int mb = 0; mb < 4; ++mb) {
                        if (mb < ncb) {
                            dmfma4 u = y[mb];
#pragma unroll
                            for (int kb = 0; kb < mb; ++kb)
#pragma unroll
                                for (int r = 0; r < 4; ++r) {
                                    const double lv = Ls[(16 * mb + ln) * CH_VP + 16 * kb + 4 * r + g];
                                    u = __builtin_amdgcn_mfma_f64_16x16x4f64(-lv, y[kb][r], u, 0, 0, 0);
                                }
                            dmfma4 x = dmfma4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const double zv = VZs[(16 * mb + ln) * CH_VP + 16 * mb + 4 * r + g];
                                x = __builtin_amdgcn_mfma_f64_16x16x4f64(zv, u[r], x, 0, 0, 0);
                            }
                            y[mb] = x;
                        }
                    }
                    const int row = rt + ln;
                    if (row < R) {
#pragma unroll
                        for (int mb = 0; mb < 4; ++mb)
                            if (mb < ncb)
                                *reinterpret_cast<double4*>(Le + (size_t)row * ld + c0 + 16 * mb +
                                                            cq) =
                                    double4{y[mb][0], y[mb][1], y[mb][2], y[mb][3]};
                    }
                    if (a.single && rt == Np) {
                        // rows Np (lanes ln == 0) and Np + 1 (ln == 1): accumulate y . z
                        double part = 0.0;
#pragma unroll
                        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const double other = __shfl_down(y[mb][r], 1, 64);
                                part = fma(y[mb][r], other, part);
                            }
                        part = ln == 0 ? part : 0.0;
                        part += __shfl_xor(part, 16, 64);
                        part += __shfl_xor(part, 32, 64);
                        if (lane == 0) dot_acc += part;
                    }
                }
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        if (bad_flag) atomicOr(a.status, MCNEGF_FLAG_NOTSPD);
        if (a.single) {
            const double* ld_ = a.lead + (size_t)e * MCNEGF_LEAD_NTERMS;
            const double tqp = a.inject_lead == 0 ? ld_[MCNEGF_LEAD_TRL] : ld_[MCNEGF_LEAD_TLR];
            const double Tk = tqp + dot_acc;
            a.T[e] = Tk;
            a.sig[e] = 0.0;
            if (!isfinite(Tk)) atomicOr(a.status, MCNEGF_FLAG_NONFINITE);
        }
    }
}

// T_k = T_qp + (row Np of L) . (row Np + 1 of L) after a factorization in several launches
// (fixed-order sum; both rows carry the same column permutation).
__global__ void __launch_bounds__(256) direct_dot_kernel(CholArgs a) {
    __shared__ double red[256];
    const int e = blockIdx.x;
    const int Np = a.Np;
    const double* Le = a.Lall + (size_t)e * (Np + 2) * a.ld;
    const double* y = Le + (size_t)Np * a.ld;
    const double* z = y + a.ld;
    double part = 0.0;
    for (int j = threadIdx.x; j < Np; j += 256) part = fma(y[j], z[j], part);
    const double dot = block_reduce256(part, red);
    if (threadIdx.x == 0) {
        const double* ld_ = a.lead + (size_t)e * MCNEGF_LEAD_NTERMS;
        const double tqp = a.inject_lead == 0 ? ld_[MCNEGF_LEAD_TRL] : ld_[MCNEGF_LEAD_TLR];
        const double Tk = tqp + dot;
        a.T[e] = Tk;
        a.sig[e] = 0.0;
        if (!isfinite(Tk)) atomicOr(a.status, MCNEGF_FLAG_NONFINITE);
    }
}

// d_I_sigma[0] = I, d_I_sigma[1] = sqrt(sum_k w_k^2 sigma_k^2), from the weighted sums.
__global__ void current_out_kernel(const double* __restrict__ reduce, double* __restrict__ out) {
    if (threadIdx.x == 0) {
        out[0] = reduce[0];
        out[1] = sqrt(reduce[1] > 0.0 ? reduce[1] : 0.0);
    }
}

hipError_t launch_current_out(const mcnegf_kernel& k, double* d_I_sigma, hipStream_t s) {
    {
        MCNEGF_TIMED("current_out_kernel", s);
        hipLaunchKernelGGL(current_out_kernel, dim3(1), dim3(64), 0, s, k.reduce, d_I_sigma);
    }
    return hipGetLastError();
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
    CholArgs a;
    a.P = k.P;
    a.vec = k.direct_vec;
    a.lead = k.lead;
    a.Lall = k.direct;
    a.T = T;
    a.sig = sigmaT;
    a.status = k.status;
    a.N = N;
    a.Np = (int)k.p_pitch;
    a.ld = k.p_pitch;
    a.inject_lead = inject_lead;
    const int nJ = (a.Np + CH_NB - 1) / CH_NB;
    // One workgroup (one CU) per energy.  When the energies leave CUs idle and the matrix is
    // large, split each energy over several workgroups, one launch per block column (the
    // launch boundary orders the block columns; no cross-workgroup waits).
    int dev = 0, cus = 0;
    if ((err = hipGetDevice(&dev)) != hipSuccess) return err;
    if ((err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
        hipSuccess)
        return err;
    // Each workgroup of an energy forms the diagonal factor itself, so keep at least two
    // super-tiles of the first block column per workgroup (four workgroups at any size).
    const int nst = (a.Np - CH_NB + CH_ROWS - 1) / CH_ROWS;
    const int cap = (nst + 1) / 2 > 4 ? (nst + 1) / 2 : 4;
    int nsplit = cus / (k.nE > 0 ? k.nE : 1);
    nsplit = nsplit > cap ? cap : nsplit;
    if (a.Np < 1024 || nJ < 4) nsplit = 1;
    if (nsplit <= 1) {
        a.J0 = 0;
        a.J1 = nJ;
        a.nsplit = 1;
        a.single = true;
        {
            MCNEGF_TIMED("cholesky_kernel", s);
            hipLaunchKernelGGL(cholesky_kernel, dim3(k.nE), dim3(64 * CH_WAVES), 0, s, a);
        }
        if ((err = hipGetLastError()) != hipSuccess) return err;
    } else {
        a.nsplit = nsplit;
        a.single = false;
        for (int J = 0; J < nJ; ++J) {
            a.J0 = J;
            a.J1 = J + 1;
            {
                MCNEGF_TIMED("cholesky_kernel", s);
                hipLaunchKernelGGL(cholesky_kernel, dim3(k.nE * nsplit), dim3(64 * CH_WAVES), 0, s,
                                   a);
            }
            if ((err = hipGetLastError()) != hipSuccess) return err;
        }
        {
            MCNEGF_TIMED("direct_dot_kernel", s);
            hipLaunchKernelGGL(direct_dot_kernel, dim3(k.nE), dim3(256), 0, s, a);
        }
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    {
        MCNEGF_TIMED("current_sum_kernel", s);
        hipLaunchKernelGGL(current_sum_kernel, dim3(1), dim3(256), 0, s, T, sigmaT, weights, k.nE,
                           k.reduce);
    }
    return hipGetLastError();
}

}  // namespace mcnegf
