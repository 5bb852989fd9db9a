// Block-tridiagonal recursive Green's functions (Sec. III B: G^r by the RGF algorithm;
// G^r = (E - H - Sigma^r)^{-1}, Sec. II A, Eq. (7)).
//
// With slices k = 0..L-1 of W sites, the diagonal blocks of E - H - Sigma are
//   A_k = E - H_kk - Sigma_B,kk - [k = 0] Sigma_L - [k = L-1] Sigma_R,
// H_kk = tridiag(-t, V, -t) and Sigma_B = diag(-(i/2) gamma) (Sec. III A, Eq. (77)); the
// off-diagonal blocks are t I (H_{k,k+1} = -t I).  Hence
//   left-connected   gL_0 = A_0^{-1},       gL_k = (A_k - t^2 gL_{k-1})^{-1},
//   right-connected  gR_{L-1} = A_{L-1}^{-1}, gR_k = (A_k - t^2 gR_{k+1})^{-1},
//   diagonal         G_kk = (A_k - t^2 gL_{k-1} - t^2 gR_{k+1})^{-1}.
// The two sweeps are sequential over slices and run as one wavefront per (energy,
// direction); the diagonal blocks are then independent and run as one wavefront each.
//
// Block inverse on one wavefront (W <= 16): the augmented [X | I] is spread over the 64 lanes,
// lane l = i + 16 q holding row i at the columns j = q + 4 m (m < M = (2W + 3) / 4).
// Gauss-Jordan elimination with partial pivoting chooses, at column p, the not-yet-used row of
// largest |x_ip| (ties: lowest row); rows are never swapped, so at the end row i holds row r_i
// of X^{-1}, r_i being the column it was pivot for.  Each lane updates its own M entries, so a
// pivot step costs a few cross-lane reads and M complex multiply-adds per lane.
#include "common.h"

namespace mcnegf {

template <int W>
struct Narrow {
    static constexpr int M = (2 * W + 3) / 4;  // entries per lane
};

// One step of an argmax over each row of 16 lanes: compare with the lane CTRL rotates in
// (DPP row_ror); every lane must be active.
template <int CTRL>
__device__ inline void argmax_step(double& mag, int& idx) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(mag), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(mag), CTRL, 0xF, 0xF, false);
    const int oi = __builtin_amdgcn_mov_dpp(idx, CTRL, 0xF, 0xF, false);
    const double om = __hiloint2double(hi, lo);
    const bool take = (om > mag) | ((om == mag) & (oi < idx));  // no short-circuit branches
    mag = take ? om : mag;
    idx = take ? oi : idx;
}
// Index of the largest mag in each row of 16 lanes (ties: lowest index), in every lane of it:
// rotations by 8, 4, 2, 1 combine all 16 values under a total order.
__device__ inline int argmax_row16(double mag, int idx) {
    argmax_step<0x128>(mag, idx);  // row_ror:8
    argmax_step<0x124>(mag, idx);  // row_ror:4
    argmax_step<0x122>(mag, idx);  // row_ror:2
    argmax_step<0x121>(mag, idx);  // row_ror:1
    return idx;
}

__device__ inline double2 shfl_c(double2 v, int src) {
    return cmk(__shfl(v.x, src, 64), __shfl(v.y, src, 64));
}
__device__ inline double readlane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Inverts the W x W matrix X held as described above (row i < W of [X | I]; rows >= W zero).
// On return row i's entries at columns W + c are (X^{-1})[rank][c].  Returns false when a
// pivot is zero or not finite.  Every lane of the wavefront must be active.
template <int W>
__device__ inline bool gj_invert(double2 (&a)[Narrow<W>::M], int i, int q, int& rank) {
    constexpr int M = Narrow<W>::M;
    bool used = i >= W;
    bool ok = true;
    rank = 0;
    // fully unrolled: the column index p selects registers, never a memory array
#pragma clang loop unroll(full)
    for (int p = 0; p < W; ++p) {
        const int qp = p & 3, mp = p >> 2;  // column p: lanes of group qp, entry mp
        const double mag = used ? -1.0 : cabs2(a[mp]);
        const int r = __builtin_amdgcn_readlane(argmax_row16(mag, i), 16 * qp);
        // the pivot row's entries at this lane's columns, and this row's entry in column p
        double2 piv[M];
#pragma unroll
        for (int m = 0; m < M; ++m) piv[m] = shfl_c(a[m], r + 16 * q);
        const double2 f = shfl_c(a[mp], i + 16 * qp);
        const double2 pp = cmk(readlane_d(a[mp].x, r + 16 * qp), readlane_d(a[mp].y, r + 16 * qp));
        const double pm = cabs2(pp);
        if (!(pm > 0.0) || !isfinite(pm)) ok = false;
        // 1 / pp = conj(pp) / |pp|^2: the reciprocal of |pp|^2 is on the pivot step's critical
        // path, so it is the hardware estimate refined by two Newton steps (each doubles the
        // correct bits) rather than a full division, a shorter dependent chain
        double rpm = __builtin_amdgcn_rcp(pm);
        rpm = fma(rpm, fma(-pm, rpm, 1.0), rpm);
        rpm = fma(rpm, fma(-pm, rpm, 1.0), rpm);
        const double2 pinv = cmk(pp.x * rpm, -pp.y * rpm);
        // per-lane choices as selects: every lane stays active for the next pivot's cross-lane
        // reads
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int j = q + 4 * m;
            const double2 pj = cmul(piv[m], pinv);
            double2 u = a[m];
            cfms(u, f, pj);
            // component selects (a select of whole double2 values goes through memory)
            const bool upd = j >= p && j < 2 * W, piv_row = i == r;
            a[m].x = upd ? (piv_row ? pj.x : u.x) : a[m].x;
            a[m].y = upd ? (piv_row ? pj.y : u.y) : a[m].y;
        }
        used = used || i == r;
        rank = i == r ? p : rank;
    }
    return ok;
}

// This lane's entries of row i of [A_k | I] for energy E (A_k = E - H_kk - Sigma_B,kk - the
// lead self-energy on an end slice); Vi, gi are the onsite energy and dephasing rate of site
// (k, i).
template <int W>
__device__ inline void diag_block_entries(double2 (&a)[Narrow<W>::M], int i, int q, int k, int L,
                                          double E, double t, double Vi, double gi,
                                          const double2* __restrict__ sig) {
#pragma unroll
    for (int m = 0; m < Narrow<W>::M; ++m) {
        const int j = q + 4 * m;
        double2 v = cmk(0.0, 0.0);
        if (i < W && j < W) {
            if (j == i) v = cmk(E - Vi, 0.5 * gi);
            if (j == i - 1 || j == i + 1) v = cmk(t, 0.0);
            if (k == 0) v = csub(v, sig[i * W + j]);
            if (k == L - 1) v = csub(v, sig[i * W + j]);
        } else if (i < W && j < 2 * W) {
            v = cmk(j - W == i ? 1.0 : 0.0, 0.0);
        }
        a[m] = v;
    }
}

template <int W>
__global__ void __launch_bounds__(64) rgf_sweep_kernel(const double* __restrict__ energies,
                                                       const double* __restrict__ onsite,
                                                       const double* __restrict__ gamma,
                                                       const double2* __restrict__ sigma, int L,
                                                       double t, double2* __restrict__ gL,
                                                       double2* __restrict__ gR,
                                                       uint32_t* __restrict__ status) {
    constexpr int M = Narrow<W>::M;
    const int e = blockIdx.x >> 1;
    const int dir = blockIdx.x & 1;
    const int lane = threadIdx.x;
    const int i = lane & 15, q = lane >> 4;
    __shared__ double2 prev[W][W];
    const double E = energies[e];
    const double2* sig = sigma + (size_t)e * W * W;
    double2* out = (dir == 0 ? gL : gR) + (size_t)e * L * W * W;
    const double t2 = t * t;
    bool ok = true;
    // the onsite energy and dephasing rate of this lane's site, loaded one slice ahead
    const int i_site = i < W ? i : 0;
    const int k_first = dir == 0 ? 0 : L - 1;
    double Vn = onsite[k_first * W + i_site], gn = gamma[k_first * W + i_site];
    for (int s = 0; s < L; ++s) {
        const int k = dir == 0 ? s : L - 1 - s;
        const double Vi = Vn, gi = gn;
        if (s + 1 < L) {
            const int kn = dir == 0 ? s + 1 : L - 2 - s;
            Vn = onsite[kn * W + i_site];
            gn = gamma[kn * W + i_site];
        }
        double2 a[M];
        diag_block_entries<W>(a, i, q, k, L, E, t, Vi, gi, sig);
        if (s > 0 && i < W) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int j = q + 4 * m;
                if (j < W) a[m] = csub(a[m], cscale(prev[i][j], t2));
            }
        }
        __syncthreads();
        int rank;
        ok &= gj_invert<W>(a, i, q, rank);
        if (i < W) {
            double2* o = out + (size_t)k * W * W + rank * W;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int j = q + 4 * m;
                if (j >= W && j < 2 * W) {
                    prev[rank][j - W] = a[m];
                    o[j - W] = a[m];
                }
            }
        }
        __syncthreads();
    }
    if (!ok && lane == 0) atomicOr(status, MCNEGF_FLAG_SINGULAR);
}

template <int W>
__global__ void __launch_bounds__(64) rgf_diag_kernel(const double* __restrict__ energies,
                                                      const double* __restrict__ onsite,
                                                      const double* __restrict__ gamma,
                                                      const double2* __restrict__ sigma, int L,
                                                      double t, const double2* __restrict__ gL,
                                                      const double2* __restrict__ gR,
                                                      double2* __restrict__ Gd,
                                                      double* __restrict__ Adiag,
                                                      uint32_t* __restrict__ status) {
    constexpr int M = Narrow<W>::M;
    const int e = blockIdx.x / L;
    const int k = blockIdx.x % L;
    const int lane = threadIdx.x;
    const int i = lane & 15, q = lane >> 4;
    const double E = energies[e];
    const double t2 = t * t;
    const int i_site = i < W ? i : 0;
    double2 a[M];
    diag_block_entries<W>(a, i, q, k, L, E, t, onsite[k * W + i_site], gamma[k * W + i_site],
                          sigma + (size_t)e * W * W);
    if (i < W) {
        const size_t base = (size_t)e * L * W * W;
        if (k > 0) {
            const double2* g = gL + base + (size_t)(k - 1) * W * W + i * W;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int j = q + 4 * m;
                if (j < W) a[m] = csub(a[m], cscale(g[j], t2));
            }
        }
        if (k < L - 1) {
            const double2* g = gR + base + (size_t)(k + 1) * W * W + i * W;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int j = q + 4 * m;
                if (j < W) a[m] = csub(a[m], cscale(g[j], t2));
            }
        }
    }
    int rank;
    const bool ok = gj_invert<W>(a, i, q, rank);
    if (i < W) {
        double2* o = Gd + ((size_t)e * L + k) * W * W + rank * W;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int j = q + 4 * m;
            if (j >= W && j < 2 * W) {
                o[j - W] = a[m];
                // the diagonal element (rank, rank) of the inverse
                if (j - W == rank) Adiag[(size_t)e * L * W + k * W + rank] = -2.0 * a[m].y;
            }
        }
    }
    if (!ok && lane == 0) atomicOr(status, MCNEGF_FLAG_SINGULAR);
}

template <int W>
static hipError_t launch_rgf_w(const mcnegf_kernel& k, const double* onsite, hipStream_t s) {
    const double2* sig = reinterpret_cast<const double2*>(k.sigma);
    double2* gL = reinterpret_cast<double2*>(k.gL);
    double2* gR = reinterpret_cast<double2*>(k.gR);
    {
        MCNEGF_TIMED("rgf_sweep_kernel", s);
        hipLaunchKernelGGL(rgf_sweep_kernel<W>, dim3(2 * k.nE), dim3(64), 0, s, k.energies, onsite,
                           k.gamma, sig, k.L, k.t, gL, gR, k.status);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    {
        MCNEGF_TIMED("rgf_diag_kernel", s);
        hipLaunchKernelGGL(rgf_diag_kernel<W>, dim3(k.nE * k.L), dim3(64), 0, s, k.energies,
                           onsite, k.gamma, sig, k.L, k.t, gL, gR,
                           reinterpret_cast<double2*>(k.Gd), k.Adiag, k.status);
    }
    return hipGetLastError();
}

// ---- wide blocks (16 < W <= 32): Gauss-Jordan with one lane per column -----------------
//
// Lane j < 2W holds column j of the augmented [X | I] (W complex values in registers, indexed
// statically).  For pivot column p, lane p picks the not-yet-used row r of largest |x_rp|
// (ties: lowest row) and writes its column to LDS; every lane scales its row-r element by
// 1 / x_rp and eliminates the other rows with the broadcast column.  Rows are never swapped:
// row p of X^{-1} is row r_p of the right half at the end, read back through LDS.

struct WideLds {
    double2 colp[32];          // pivot column
    double2 full[32][65];      // all columns at the end (row-major, padded)
    int prow[32];              // pivot row of each column
};

// col[r] for a uniform r, as a masked sum (a select chain here would be folded into a
// dynamic index, which moves the whole column to scratch memory).
template <int W>
__device__ inline double2 select_row(const double2 (&col)[W], int r) {
    double2 v = cmk(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const double m = (double)(i == r);
        v.x = fma(col[i].x, m, v.x);
        v.y = fma(col[i].y, m, v.y);
    }
    return v;
}

// Inverts the matrix whose column j < W is col[] of lane j (lanes W..2W-1 start as the
// identity columns); afterwards S.full[i][W + x] = (right half)[i][x] and S.prow[p] = r_p, so
// (X^{-1})[p][x] = S.full[S.prow[p]][W + x].  Returns false on a zero or non-finite pivot.
template <int W>
__device__ inline bool gj_invert_wide(double2 (&col)[W], int lane, WideLds& S) {
    uint32_t used = 0u;
    bool ok = true;
    for (int p = 0; p < W; ++p) {  // uniform loop
        int r = 0;
        if (lane == p) {  // divergent region: the owner of column p searches it
            double best = -1.0;
#pragma unroll
            for (int i = 0; i < W; ++i) {
                const double m = cabs2(col[i]);
                if (!((used >> i) & 1u) && m > best) {
                    best = m;
                    r = i;
                }
            }
#pragma unroll
            for (int i = 0; i < W; ++i) S.colp[i] = col[i];
        }
        r = __builtin_amdgcn_readlane(r, p);
        __syncthreads();
        const double2 piv = S.colp[r];
        const double pm = cabs2(piv);
        if (!(pm > 0.0) || !isfinite(pm)) ok = false;
        const double2 pinv = crecip(piv);
        const double2 sr = cmul(select_row<W>(col, r), pinv);
#pragma unroll
        for (int i = 0; i < W; ++i) {
            // row r takes sr, every other row i subtracts x_ip sr (x_rp sr = sr for row r)
            const double keep = (double)(i != r);
            const double2 cip = S.colp[i];
            double2 v = col[i];
            cfms(v, cip, sr);
            col[i] = cmk(fma(keep, v.x - sr.x, sr.x), fma(keep, v.y - sr.y, sr.y));
        }
        used |= 1u << r;
        if (lane == 0) S.prow[p] = r;
        __syncthreads();  // colp is rewritten for the next pivot
    }
    if (lane < 2 * W) {
#pragma unroll
        for (int i = 0; i < W; ++i) S.full[i][lane] = col[i];
    }
    __syncthreads();
    return ok;
}

// Column j (lane j < W) of A_k, or the identity column j - W (lanes W .. 2W-1).
template <int W>
__device__ inline void diag_block_col(double2 (&col)[W], int j, int k, int L, double E, double t,
                                      const double* __restrict__ onsite,
                                      const double* __restrict__ gamma,
                                      const double2* __restrict__ sig) {
#pragma unroll
    for (int i = 0; i < W; ++i) {
        double2 v = cmk(0.0, 0.0);
        if (j < W) {
            if (i == j) v = cmk(E - onsite[k * W + i], 0.5 * gamma[k * W + i]);
            if (i == j - 1 || i == j + 1) v = cmk(t, 0.0);
            if (k == 0) v = csub(v, sig[i * W + j]);
            if (k == L - 1) v = csub(v, sig[i * W + j]);
        } else if (j < 2 * W) {
            v = cmk(i == j - W ? 1.0 : 0.0, 0.0);
        }
        col[i] = v;
    }
}

template <int W>
__global__ void __launch_bounds__(64) rgf_sweep_wide_kernel(const double* __restrict__ energies,
                                                            const double* __restrict__ onsite,
                                                            const double* __restrict__ gamma,
                                                            const double2* __restrict__ sigma,
                                                            int L, double t,
                                                            double2* __restrict__ gL,
                                                            double2* __restrict__ gR,
                                                            uint32_t* __restrict__ status) {
    __shared__ WideLds S;
    __shared__ double2 prev[W][W + 1];
    const int e = blockIdx.x >> 1;
    const int dir = blockIdx.x & 1;
    const int lane = threadIdx.x;
    const double E = energies[e];
    const double2* sig = sigma + (size_t)e * W * W;
    double2* out = (dir == 0 ? gL : gR) + (size_t)e * L * W * W;
    const double t2 = t * t;
    bool ok = true;
    for (int s = 0; s < L; ++s) {
        const int k = dir == 0 ? s : L - 1 - s;
        double2 col[W];
        const int j = lane < 2 * W ? lane : 2 * W;
        diag_block_col<W>(col, j, k, L, E, t, onsite, gamma, sig);
        if (s > 0 && lane < W) {
#pragma unroll
            for (int i = 0; i < W; ++i) col[i] = csub(col[i], cscale(prev[i][lane], t2));
        }
        ok &= gj_invert_wide<W>(col, lane, S);
        // row p of the inverse: lane x < W writes element (p, x)
        if (lane < W) {
            double2* o = out + (size_t)k * W * W;
            for (int p = 0; p < W; ++p) {
                const double2 v = S.full[S.prow[p]][W + lane];
                prev[p][lane] = v;
                o[p * W + lane] = v;
            }
        }
        __syncthreads();
    }
    if (!ok && lane == 0) atomicOr(status, MCNEGF_FLAG_SINGULAR);
}

template <int W>
__global__ void __launch_bounds__(64) rgf_diag_wide_kernel(const double* __restrict__ energies,
                                                           const double* __restrict__ onsite,
                                                           const double* __restrict__ gamma,
                                                           const double2* __restrict__ sigma,
                                                           int L, double t,
                                                           const double2* __restrict__ gL,
                                                           const double2* __restrict__ gR,
                                                           double2* __restrict__ Gd,
                                                           double* __restrict__ Adiag,
                                                           uint32_t* __restrict__ status) {
    __shared__ WideLds S;
    const int e = blockIdx.x / L;
    const int k = blockIdx.x % L;
    const int lane = threadIdx.x;
    const double E = energies[e];
    const double t2 = t * t;
    double2 col[W];
    const int j = lane < 2 * W ? lane : 2 * W;
    diag_block_col<W>(col, j, k, L, E, t, onsite, gamma, sigma + (size_t)e * W * W);
    if (lane < W) {
        const size_t base = (size_t)e * L * W * W;
        if (k > 0) {
            const double2* g = gL + base + (size_t)(k - 1) * W * W;
#pragma unroll
            for (int i = 0; i < W; ++i) col[i] = csub(col[i], cscale(g[i * W + lane], t2));
        }
        if (k < L - 1) {
            const double2* g = gR + base + (size_t)(k + 1) * W * W;
#pragma unroll
            for (int i = 0; i < W; ++i) col[i] = csub(col[i], cscale(g[i * W + lane], t2));
        }
    }
    const bool ok = gj_invert_wide<W>(col, lane, S);
    if (lane < W) {
        double2* o = Gd + ((size_t)e * L + k) * W * W;
        for (int p = 0; p < W; ++p) o[p * W + lane] = S.full[S.prow[p]][W + lane];
        // diagonal element (x, x) of the inverse for x = lane
        Adiag[(size_t)e * L * W + k * W + lane] = -2.0 * S.full[S.prow[lane]][W + lane].y;
    }
    if (!ok && lane == 0) atomicOr(status, MCNEGF_FLAG_SINGULAR);
}

// ---- wide sweeps on a workgroup: one (energy, direction) chain per 256 threads ----------
//
// The W x W block (padded to 32 x 32 with the identity) is spread over four wavefronts: lane
// l of wavefront w holds column c = 8 w + (l >> 3) at rows 4 (l & 7) + s, s = 0..3.  The block
// is inverted in place by Gauss-Jordan exchange steps with the same pivot rule as above (at
// column p, the not-yet-used row r of largest |x_rp|, lowest row on ties): with pinv = 1/x_rp,
//   x_rc <- x_rc pinv (c != p),  x_rp <- pinv,
//   x_ic <- x_ic - x_ip x_rc pinv (i != r, c != p),  x_ip <- -x_ip pinv (i != r).
// After the W steps the stored Y holds the inverse with rows and columns permuted: with
// pi(p) = r_p, (X^{-1})[p][q] = Y[pi(p)][pi^{-1}(q)].  Column p of each step reaches every
// thread through LDS (written by its owners at the end of step p - 1, double-buffered: one
// barrier per step); the pivot row's entry x_rc is in the same wavefront and is read with a
// lane shuffle.  Every thread computes the same pivot from the same LDS column.

// Complex arithmetic in the sweep's precision: C = double2 (FP64) or float2 (FP32 sweeps of a
// build with FP32 block products; the blocks are stored in FP64 either way).
__device__ inline float2 cmk_t(float re, float im, float2) { return make_float2(re, im); }
__device__ inline double2 cmk_t(double re, double im, double2) { return cmk(re, im); }
__device__ inline float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }
__device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline void cfms(float2& a, float2 b, float2 c) {
    a.x = fmaf(-b.x, c.x, fmaf(b.y, c.y, a.x));
    a.y = fmaf(-b.x, c.y, fmaf(-b.y, c.x, a.y));
}
__device__ inline float2 crecip(float2 a) {
    if (fabsf(a.x) >= fabsf(a.y)) {
        const float r = a.y / a.x, d = a.x + a.y * r;
        return make_float2(1.0f / d, -r / d);
    }
    const float r = a.x / a.y, d = a.y + a.x * r;
    return make_float2(r / d, -1.0f / d);
}

template <typename C>
struct WgLds {
    C col[2][32];   // pivot column of the current step, double-buffered
    C y[32][33];    // the permuted inverse, gathered at the end of a slice
    int perm[32];   // perm[p] = r_p
    int iperm[32];  // iperm[r_p] = p
};

template <int W, typename C = double2>
__global__ void __launch_bounds__(256) rgf_sweep_wg_kernel(const double* __restrict__ energies,
                                                           const double* __restrict__ onsite,
                                                           const double* __restrict__ gamma,
                                                           const double2* __restrict__ sigma,
                                                           int L, double t,
                                                           double2* __restrict__ gL,
                                                           double2* __restrict__ gR,
                                                           uint32_t* __restrict__ status) {
    typedef decltype(C().x) R;  // real type of the sweep
    __shared__ WgLds<C> S;
    const int e = blockIdx.x >> 1;
    const int dir = blockIdx.x & 1;
    const int lane = threadIdx.x & 63;
    const int c = 8 * (threadIdx.x >> 6) + (lane >> 3);  // this thread's column
    const int rg = lane & 7;                              // rows 4 rg .. 4 rg + 3
    const double E = energies[e];
    const double2* sig = sigma + (size_t)e * W * W;
    double2* out = (dir == 0 ? gL : gR) + (size_t)e * L * W * W;
    const double t2 = t * t;
    bool ok = true;
    C gprev[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) gprev[s] = cmk_t((R)0, (R)0, C());
    // onsite energy and dephasing rate of site (k, c), loaded one slice ahead
    const int cs = c < W ? c : 0;
    const int k_first = dir == 0 ? 0 : L - 1;
    double Vn = onsite[k_first * W + cs], gn = gamma[k_first * W + cs];
    for (int sl = 0; sl < L; ++sl) {
        const int k = dir == 0 ? sl : L - 1 - sl;
        const double Vc = Vn, gc = gn;
        if (sl + 1 < L) {
            const int kn = dir == 0 ? sl + 1 : L - 2 - sl;
            Vn = onsite[kn * W + cs];
            gn = gamma[kn * W + cs];
        }
        // this thread's entries of X = A_k - t^2 g_{k-1} (identity outside W x W)
        C a[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int i = 4 * rg + s;
            double2 v = cmk(i == c ? 1.0 : 0.0, 0.0);
            if (i < W && c < W) {
                v = cmk(0.0, 0.0);
                if (i == c) v = cmk(E - Vc, 0.5 * gc);
                if (i == c - 1 || i == c + 1) v = cmk(t, 0.0);
                if (k == 0) v = csub(v, sig[i * W + c]);
                if (k == L - 1) v = csub(v, sig[i * W + c]);
            }
            C u = cmk_t((R)v.x, (R)v.y, C());
            if (i < W && c < W && sl > 0) {
                u.x -= (R)t2 * gprev[s].x;
                u.y -= (R)t2 * gprev[s].y;
            }
            a[s] = u;
        }
        if (c == 0) {
#pragma unroll
            for (int s = 0; s < 4; ++s) S.col[0][4 * rg + s] = a[s];
        }
        __syncthreads();
        uint32_t used = 0u;
        for (int p = 0; p < W; ++p) {  // uniform loop
            const C* cb = S.col[p & 1];
            C f[4];
            R best = (R)-1;
            int bi = 64;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int i = 4 * rg + s;
                f[s] = cb[i];
                const R m = (i < W && !((used >> i) & 1u)) ? cabs2(f[s]) : (R)-1;
                const bool take = m > best;  // rows in increasing order: ties keep the lower
                best = take ? m : best;
                bi = take ? i : bi;
            }
            // argmax over the 8 lanes of this column's group (ties: lowest row)
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) {
                const R ob = __shfl_xor(best, o, 64);
                const int oi = __shfl_xor(bi, o, 64);
                const bool take = (ob > best) | ((ob == best) & (oi < bi));
                best = take ? ob : best;
                bi = take ? oi : bi;
            }
            int r = __builtin_amdgcn_readfirstlane(bi);
            if (r >= W) {  // no finite candidate (NaN entries): flag it, keep indices in range
                r = __builtin_ctz(~used);
                ok = false;
            }
            const C pv = cb[r];
            const R pm = cabs2(pv);
            if (!(pm > (R)0) || !isfinite(pm)) ok = false;
            const C pinv = crecip(pv);
            // x_rc from the lane holding row r of this column
            // a[r & 3] as a masked sum (a select chain would become a dynamic index into
            // scratch memory)
            const int rs = r & 3;
            C own = cmk_t((R)0, (R)0, C());
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const R m = (R)(s == rs);
                own.x = fma(a[s].x, m, own.x);
                own.y = fma(a[s].y, m, own.y);
            }
            const int src = (lane & ~7) | (r >> 2);
            const C xrc = cmk_t(__shfl(own.x, src, 64), __shfl(own.y, src, 64), C());
            const C q = cmul(xrc, pinv);
            const bool piv_col = c == p;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int i = 4 * rg + s;
                const bool piv_row = i == r;
                C u = a[s];
                cfms(u, f[s], q);                 // x_ic - x_ip x_rc pinv
                const C wcol = cmul(f[s], pinv);  // x_ip pinv
                C v;
                v.x = piv_col ? (piv_row ? pinv.x : -wcol.x) : (piv_row ? q.x : u.x);
                v.y = piv_col ? (piv_row ? pinv.y : -wcol.y) : (piv_row ? q.y : u.y);
                a[s] = v;
            }
            used |= 1u << r;
            if (threadIdx.x == 0) {
                S.perm[p] = r;
                S.iperm[r] = p;
            }
            if (c == p + 1) {
#pragma unroll
                for (int s = 0; s < 4; ++s) S.col[(p + 1) & 1][4 * rg + s] = a[s];
            }
            __syncthreads();
        }
        // gather g_k = X^{-1}: entry (i, c) = Y[perm[i]][iperm[c]]
#pragma unroll
        for (int s = 0; s < 4; ++s) S.y[4 * rg + s][c] = a[s];
        __syncthreads();
        if (c < W) {
            const int jc = S.iperm[c];
            double2* o = out + (size_t)k * W * W;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int i = 4 * rg + s;
                if (i < W) {
                    const C v = S.y[S.perm[i]][jc];
                    gprev[s] = v;
                    o[i * W + c] = cmk((double)v.x, (double)v.y);
                }
            }
        }
        // S.col[0] is written next at the start of the next slice, after these reads of S.y,
        // S.perm and S.iperm; they are rewritten only after the next slice's first barrier
    }
    if (!ok && threadIdx.x == 0) atomicOr(status, MCNEGF_FLAG_SINGULAR);
}

// The left/right sweeps on a workgroup per chain, in FP64 or (fp32) in FP32.
template <int W>
static hipError_t launch_rgf_sweep_wg(const mcnegf_kernel& k, const double* onsite, bool fp32,
                                      hipStream_t s) {
    const double2* sig = reinterpret_cast<const double2*>(k.sigma);
    double2* gL = reinterpret_cast<double2*>(k.gL);
    double2* gR = reinterpret_cast<double2*>(k.gR);
    MCNEGF_TIMED("rgf_sweep_kernel", s);
    if (fp32)
        hipLaunchKernelGGL((rgf_sweep_wg_kernel<W, float2>), dim3(2 * k.nE), dim3(256), 0, s,
                           k.energies, onsite, k.gamma, sig, k.L, k.t, gL, gR, k.status);
    else
        hipLaunchKernelGGL((rgf_sweep_wg_kernel<W, double2>), dim3(2 * k.nE), dim3(256), 0, s,
                           k.energies, onsite, k.gamma, sig, k.L, k.t, gL, gR, k.status);
    return hipGetLastError();
}

template <int W>
static hipError_t launch_rgf_wide(const mcnegf_kernel& k, const double* onsite, hipStream_t s) {
    const double2* sig = reinterpret_cast<const double2*>(k.sigma);
    double2* gL = reinterpret_cast<double2*>(k.gL);
    double2* gR = reinterpret_cast<double2*>(k.gR);
    if (launch_rgf_sweep_wg<W>(k, onsite, false, s) != hipSuccess) return hipGetLastError();
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    {
        MCNEGF_TIMED("rgf_diag_kernel", s);
        hipLaunchKernelGGL(rgf_diag_wide_kernel<W>, dim3(k.nE * k.L), dim3(64), 0, s, k.energies,
                           onsite, k.gamma, sig, k.L, k.t, gL, gR,
                           reinterpret_cast<double2*>(k.Gd), k.Adiag, k.status);
    }
    return hipGetLastError();
}

// FP32 sweeps (a build with FP32 block products, W = 16 or 32), then the FP64 diagonal blocks.
hipError_t launch_rgf_fp32(const mcnegf_kernel& k, const double* onsite, hipStream_t s) {
    const double2* sig = reinterpret_cast<const double2*>(k.sigma);
    const double2* gL = reinterpret_cast<const double2*>(k.gL);
    const double2* gR = reinterpret_cast<const double2*>(k.gR);
    hipError_t err;
    if (k.W == 16) {
        if ((err = launch_rgf_sweep_wg<16>(k, onsite, true, s)) != hipSuccess) return err;
        MCNEGF_TIMED("rgf_diag_kernel", s);
        hipLaunchKernelGGL(rgf_diag_kernel<16>, dim3(k.nE * k.L), dim3(64), 0, s, k.energies,
                           onsite, k.gamma, sig, k.L, k.t, gL, gR,
                           reinterpret_cast<double2*>(k.Gd), k.Adiag, k.status);
        return hipGetLastError();
    }
    if (k.W == 32) {
        if ((err = launch_rgf_sweep_wg<32>(k, onsite, true, s)) != hipSuccess) return err;
        MCNEGF_TIMED("rgf_diag_kernel", s);
        hipLaunchKernelGGL(rgf_diag_wide_kernel<32>, dim3(k.nE * k.L), dim3(64), 0, s,
                           k.energies, onsite, k.gamma, sig, k.L, k.t, gL, gR,
                           reinterpret_cast<double2*>(k.Gd), k.Adiag, k.status);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

hipError_t launch_rgf(const mcnegf_kernel& k, const double* onsite, hipStream_t s) {
    switch (k.W) {
#define MCNEGF_CASE(w) \
    case w:            \
        return launch_rgf_w<w>(k, onsite, s);
        MCNEGF_CASE(1) MCNEGF_CASE(2) MCNEGF_CASE(3) MCNEGF_CASE(4) MCNEGF_CASE(5)
        MCNEGF_CASE(6) MCNEGF_CASE(7) MCNEGF_CASE(8) MCNEGF_CASE(9) MCNEGF_CASE(10)
        MCNEGF_CASE(11) MCNEGF_CASE(12) MCNEGF_CASE(13) MCNEGF_CASE(14) MCNEGF_CASE(15)
        MCNEGF_CASE(16)
#undef MCNEGF_CASE
#define MCNEGF_WIDE(w) \
    case w:            \
        return launch_rgf_wide<w>(k, onsite, s);
        MCNEGF_WIDE(17) MCNEGF_WIDE(18) MCNEGF_WIDE(19) MCNEGF_WIDE(20) MCNEGF_WIDE(21)
        MCNEGF_WIDE(22) MCNEGF_WIDE(23) MCNEGF_WIDE(24) MCNEGF_WIDE(25) MCNEGF_WIDE(26)
        MCNEGF_WIDE(27) MCNEGF_WIDE(28) MCNEGF_WIDE(29) MCNEGF_WIDE(30) MCNEGF_WIDE(31)
        MCNEGF_WIDE(32)
#undef MCNEGF_WIDE
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace mcnegf
