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
// Block inverse on one wavefront: lane i < W holds row i of the augmented [X | I] in
// registers; Gauss-Jordan elimination with partial pivoting chooses, at column p, the
// not-yet-used row of largest |x_ip| (ties: lowest lane); rows are never swapped, so at
// the end lane i holds row r_i of X^{-1}, r_i being the column it was pivot for.
#include "common.h"

namespace mcnegf {

__device__ inline double readlane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Largest mag over lanes 0..15 (every lane of each 16-lane group gets its group's winner).
__device__ inline int argmax16(double mag, int lane) {
    int idx = lane;
#pragma unroll
    for (int off = 8; off >= 1; off >>= 1) {
        const double om = __shfl_xor(mag, off, 64);
        const int oi = __shfl_xor(idx, off, 64);
        if (om > mag || (om == mag && oi < idx)) {
            mag = om;
            idx = oi;
        }
    }
    return idx;
}

// Inverts the W x W matrix whose row i is a[0..W-1] of lane i (lanes >= W hold zeros).
// On return a[W..2W-1] of lane i is row `rank` of the inverse.  Returns false when a pivot
// is zero or not finite.
template <int W>
__device__ inline bool gj_invert(double2 (&a)[2 * W], int lane, int& rank) {
    bool used = lane >= W;
    bool ok = true;
    rank = 0;
#pragma unroll
    for (int p = 0; p < W; ++p) {
        const double mag = used ? -1.0 : cabs2(a[p]);
        const int r = __builtin_amdgcn_readfirstlane(argmax16(mag, lane));
        double2 piv[2 * W];
#pragma unroll
        for (int j = p; j < 2 * W; ++j)
            piv[j] = cmk(readlane_d(a[j].x, r), readlane_d(a[j].y, r));
        const double pm = cabs2(piv[p]);
        if (!(pm > 0.0) || !isfinite(pm)) ok = false;
        const double2 pinv = crecip(piv[p]);
#pragma unroll
        for (int j = p; j < 2 * W; ++j) piv[j] = cmul(piv[j], pinv);
        if (lane == r) {
#pragma unroll
            for (int j = p; j < 2 * W; ++j) a[j] = piv[j];
            used = true;
            rank = p;
        } else {
            const double2 f = a[p];
#pragma unroll
            for (int j = p; j < 2 * W; ++j) cfms(a[j], f, piv[j]);
        }
    }
    return ok;
}

// Row i (< W) of A_k for energy E, in a[0..W-1]; identity row in a[W..2W-1]; Vi, gi are the
// onsite energy and dephasing rate of site (k, i).
template <int W>
__device__ inline void diag_block_row_v(double2 (&a)[2 * W], int i, int k, int L, double E,
                                        double t, double Vi, double gi,
                                        const double2* __restrict__ sig) {
#pragma unroll
    for (int j = 0; j < 2 * W; ++j) a[j] = cmk(0.0, 0.0);
    if (i >= W) return;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        double2 v = cmk(0.0, 0.0);
        if (j == i) v = cmk(E - Vi, 0.5 * gi);
        if (j == i - 1 || j == i + 1) v = cmk(t, 0.0);
        if (k == 0) v = csub(v, sig[i * W + j]);
        if (k == L - 1) v = csub(v, sig[i * W + j]);
        a[j] = v;
        a[W + j] = cmk(j == i ? 1.0 : 0.0, 0.0);
    }
}

template <int W>
__device__ inline void diag_block_row(double2 (&a)[2 * W], int i, int k, int L, double E, double t,
                                      const double* __restrict__ onsite,
                                      const double* __restrict__ gamma,
                                      const double2* __restrict__ sig) {
#pragma unroll
    for (int j = 0; j < 2 * W; ++j) a[j] = cmk(0.0, 0.0);
    if (i >= W) return;
    const int site = k * W + i;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        double2 v = cmk(0.0, 0.0);
        if (j == i) v = cmk(E - onsite[site], 0.5 * gamma[site]);
        if (j == i - 1 || j == i + 1) v = cmk(t, 0.0);
        if (k == 0) v = csub(v, sig[i * W + j]);
        if (k == L - 1) v = csub(v, sig[i * W + j]);
        a[j] = v;
        a[W + j] = cmk(j == i ? 1.0 : 0.0, 0.0);
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
    const int e = blockIdx.x >> 1;
    const int dir = blockIdx.x & 1;
    const int lane = threadIdx.x;
    __shared__ double2 prev[W][W];
    const double E = energies[e];
    const double2* sig = sigma + (size_t)e * W * W;
    double2* out = (dir == 0 ? gL : gR) + (size_t)e * L * W * W;
    const double t2 = t * t;
    bool ok = true;
    // the onsite energy and dephasing rate of this lane's site, loaded one slice ahead
    const int i_site = lane < W ? lane : 0;
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
        double2 a[2 * W];
        diag_block_row_v<W>(a, lane, k, L, E, t, Vi, gi, sig);
        if (s > 0 && lane < W) {
#pragma unroll
            for (int j = 0; j < W; ++j) a[j] = csub(a[j], cscale(prev[lane][j], t2));
        }
        __syncthreads();
        int rank;
        ok &= gj_invert<W>(a, lane, rank);
        if (lane < W) {
            double2* o = out + (size_t)k * W * W + rank * W;
#pragma unroll
            for (int j = 0; j < W; ++j) {
                prev[rank][j] = a[W + j];
                o[j] = a[W + j];
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
    const int e = blockIdx.x / L;
    const int k = blockIdx.x % L;
    const int lane = threadIdx.x;
    const double E = energies[e];
    const double t2 = t * t;
    double2 a[2 * W];
    diag_block_row<W>(a, lane, k, L, E, t, onsite, gamma, sigma + (size_t)e * W * W);
    if (lane < W) {
        const size_t base = (size_t)e * L * W * W;
        if (k > 0) {
            const double2* g = gL + base + (size_t)(k - 1) * W * W + lane * W;
#pragma unroll
            for (int j = 0; j < W; ++j) a[j] = csub(a[j], cscale(g[j], t2));
        }
        if (k < L - 1) {
            const double2* g = gR + base + (size_t)(k + 1) * W * W + lane * W;
#pragma unroll
            for (int j = 0; j < W; ++j) a[j] = csub(a[j], cscale(g[j], t2));
        }
    }
    int rank;
    const bool ok = gj_invert<W>(a, lane, rank);
    if (lane < W) {
        double2* o = Gd + ((size_t)e * L + k) * W * W + rank * W;
#pragma unroll
        for (int j = 0; j < W; ++j) o[j] = a[W + j];
        // diagonal element (rank, rank): a[W + rank], selected without dynamic indexing
        double im = 0.0;
#pragma unroll
        for (int j = 0; j < W; ++j)
            if (j == rank) im = a[W + j].y;
        Adiag[(size_t)e * L * W + k * W + rank] = -2.0 * im;
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

template <int W>
static hipError_t launch_rgf_wide(const mcnegf_kernel& k, const double* onsite, hipStream_t s) {
    const double2* sig = reinterpret_cast<const double2*>(k.sigma);
    double2* gL = reinterpret_cast<double2*>(k.gL);
    double2* gR = reinterpret_cast<double2*>(k.gR);
    {
        MCNEGF_TIMED("rgf_sweep_kernel", s);
        hipLaunchKernelGGL(rgf_sweep_wide_kernel<W>, dim3(2 * k.nE), dim3(64), 0, s, k.energies,
                           onsite, k.gamma, sig, k.L, k.t, gL, gR, k.status);
    }
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
