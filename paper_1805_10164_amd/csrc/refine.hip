// One FP64 refinement step on G^r after the full inverse with FP32 block products (a build
// with MCNEGF_BUILD_FP32_PRODUCTS | MCNEGF_BUILD_FP32_REFINE).
//
// G0 (every block of G from the FP32 sweeps, stored) is corrected column by column by one
// step of mixed-precision iterative refinement of (E - H - Sigma) G = I (Sec. II A, Eq. (7)):
//   R = I - A G0 in FP64, from the 5-point stencil of A (diagonal E - V_i + (i/2) gamma_i,
//       +t to the four neighbours) and the lead self-energies on the end slices;
//   A D = R solved in FP32 with the block LU that the left-connected RGF blocks give,
//       forward  y_k = gL_k (r_k - t y_{k-1}),  backward  d_k = y_k - t gL_k d_{k+1};
//   G1 = G0 + D in FP64,
// and G1 goes straight into what the build keeps: |G1_ij|^2 (P), the exit weights
// <psi_j|Gamma_r|psi_j>, the corner and diagonal blocks and A_jj = -2 Im G1_jj.  One lane per column (a wavefront owns 64
// consecutive columns); the RGF block of each slice is staged in LDS in FP32 one slice ahead
// (double-buffered) and read by every lane at the same address.
#include "common.h"

namespace mcnegf {

typedef __attribute__((address_space(3))) float lds_float;

template <int W>
__device__ inline void stage_block_f32(lds_float* dst, const double2* __restrict__ src, int tid) {
#pragma unroll
    for (int i = tid; i < W * W; i += 64) {
        const double2 v = src[i];
        dst[2 * i] = (float)v.x;
        dst[2 * i + 1] = (float)v.y;
    }
}

// out = M in for a W x W complex block M staged as FP32 (re, im) pairs, row-major.
template <int W>
__device__ inline void matvec_f32(float2 (&out)[W], const float2 (&in)[W], const lds_float* M) {
#pragma unroll
    for (int y = 0; y < W; ++y) {
        float re = 0.0f, im = 0.0f;
#pragma unroll
        for (int x = 0; x < W; ++x) {
            const float mr = M[2 * (y * W + x)], mi = M[2 * (y * W + x) + 1];
            re = fmaf(mr, in[x].x, fmaf(-mi, in[x].y, re));
            im = fmaf(mr, in[x].y, fmaf(mi, in[x].x, im));
        }
        out[y] = make_float2(re, im);
    }
}

template <int W>
__global__ void __launch_bounds__(64) refine_kernel(
    const double2* __restrict__ gL, const double2* __restrict__ G0, float2* __restrict__ Y,
    int64_t ld, const double* __restrict__ energies, const double* __restrict__ onsite,
    const double* __restrict__ gamma, const double2* __restrict__ sigma,
    const double* __restrict__ gam_lead, int L, double t, double* __restrict__ P, int64_t ldP,
    double* __restrict__ wL, double* __restrict__ wR, double2* __restrict__ corner,
    double2* __restrict__ Gd, double* __restrict__ Adiag) {
    const int N = W * L;
    const int e = blockIdx.y;
    const int lane = threadIdx.x;
    const int c = blockIdx.x * 64 + lane;
    const bool valid = c < N;
    const int cl = valid ? c : N - 1;  // column that idle lanes read
    const int lc = cl / W, yc = cl - lc * W;
    const double E = energies[e];
    const double2* sig = sigma + (size_t)e * W * W;
    const double* gm = gam_lead + (size_t)e * W * W;
    const double2* G0e = G0 + (size_t)e * N * ld;
    float2* Ye = Y + (size_t)e * N * ld;
    const double2* gLe = gL + (size_t)e * L * W * W;
    double* Pe = P + (size_t)e * N * ldP;
    double2* cRL = corner + (size_t)e * 2 * W * W;
    double2* cLR = cRL + W * W;
    double2* Gde = Gd + ((size_t)e * L + lc) * W * W;  // diagonal block of this column's slice
    const float tf = (float)t;
    constexpr int BS = 2 * W * W;
    __shared__ float Ms_raw[2 * BS];
    __shared__ double2 endv[W][64];  // a lane's column on an end slice (exit weights)
    lds_float* Ms = (lds_float*)Ms_raw;
    auto g0 = [&](int row) -> double2 { return G0e[(size_t)row * ld + cl]; };

    // ---- forward: y_k = gL_k r_k - t gL_k y_{k-1}, with r_k = (I - A G0)_k in FP64 --------
    float2 y[W];
#pragma unroll
    for (int r = 0; r < W; ++r) y[r] = make_float2(0.0f, 0.0f);
    stage_block_f32<W>(Ms, gLe, lane);
    for (int k = 0; k < L; ++k) {
        __syncthreads();  // block k staged; the other buffer is no longer read
        const lds_float* M = Ms + (k & 1) * BS;
        if (k + 1 < L)
            stage_block_f32<W>(Ms + ((k + 1) & 1) * BS, gLe + (size_t)(k + 1) * W * W, lane);
        float2 acc[W];
        matvec_f32<W>(acc, y, M);
#pragma unroll
        for (int x = 0; x < W; ++x) acc[x] = make_float2(-tf * acc[x].x, -tf * acc[x].y);
#pragma unroll 4
        for (int r = 0; r < W; ++r) {  // residual rows, each added as column r of M
            const int i = k * W + r;
            const double2 g = g0(i);
            const double d = E - onsite[i], h = 0.5 * gamma[i];
            double2 a = cmk(d * g.x - h * g.y, d * g.y + h * g.x);
            double2 nb = cmk(0.0, 0.0);
            if (r > 0) nb = cadd(nb, g0(i - 1));
            if (r < W - 1) nb = cadd(nb, g0(i + 1));
            if (k > 0) nb = cadd(nb, g0(i - W));
            if (k < L - 1) nb = cadd(nb, g0(i + W));
            a = cadd(a, cscale(nb, t));
            if (k == 0)
                for (int q = 0; q < W; ++q) cfms(a, sig[r * W + q], g0(q));
            if (k == L - 1)
                for (int q = 0; q < W; ++q) cfms(a, sig[r * W + q], g0((L - 1) * W + q));
            const float rr = (float)((i == c ? 1.0 : 0.0) - a.x), ri = (float)(-a.y);
#pragma unroll
            for (int x = 0; x < W; ++x) {
                const float mr = M[2 * (x * W + r)], mi = M[2 * (x * W + r) + 1];
                acc[x].x = fmaf(mr, rr, fmaf(-mi, ri, acc[x].x));
                acc[x].y = fmaf(mr, ri, fmaf(mi, rr, acc[x].y));
            }
        }
#pragma unroll
        for (int r = 0; r < W; ++r) y[r] = acc[r];
        if (valid) {
#pragma unroll
            for (int r = 0; r < W; ++r) Ye[(size_t)(k * W + r) * ld + c] = y[r];
        }
    }
    // ---- backward: d_k = y_k - t gL_k d_{k+1}; G1 = G0 + d --------------------------------
    // y holds d_{L-1} = y_{L-1}
    __syncthreads();  // forward reads of both buffers done
    if (L > 1) stage_block_f32<W>(Ms, gLe + (size_t)(L - 2) * W * W, lane);
    for (int k = L - 1; k >= 0; --k) {
        if (k < L - 1) {
            const int j = L - 2 - k;
            __syncthreads();
            const lds_float* M = Ms + (j & 1) * BS;
            if (k > 0)
                stage_block_f32<W>(Ms + ((j + 1) & 1) * BS, gLe + (size_t)(k - 1) * W * W, lane);
            float2 acc[W];
            matvec_f32<W>(acc, y, M);
#pragma unroll
            for (int r = 0; r < W; ++r) {
                const float2 yk = Ye[(size_t)(k * W + r) * ld + cl];
                y[r] = make_float2(yk.x - tf * acc[r].x, yk.y - tf * acc[r].y);
            }
        }
        const bool end = k == 0 || k == L - 1;
#pragma unroll
        for (int r = 0; r < W; ++r) {
            const double2 g = g0(k * W + r);
            const double2 g1 = cmk(g.x + (double)y[r].x, g.y + (double)y[r].y);
            if (valid) Pe[(size_t)(k * W + r) * ldP + c] = g1.x * g1.x + g1.y * g1.y;
            if (end) endv[r][lane] = g1;
            if (valid && k == lc) {
                Gde[r * W + yc] = g1;
                if (r == yc) Adiag[(size_t)e * N + c] = -2.0 * g1.y;
            }
        }
        if (end && valid) {
            // Re v^+ Gamma v over the end slice, Gamma real symmetric
            double q = 0.0;
            for (int a = 0; a < W; ++a) {
                const double2 va = endv[a][lane];
                double2 u = cmk(0.0, 0.0);
                for (int b = 0; b < W; ++b) {
                    const double gab = gm[a * W + b];
                    const double2 vb = endv[b][lane];
                    u.x = fma(gab, vb.x, u.x);
                    u.y = fma(gab, vb.y, u.y);
                }
                q = fma(va.x, u.x, fma(va.y, u.y, q));
            }
            if (k == L - 1) {
                wR[(size_t)e * N + c] = q;
                if (lc == 0)  // G_{L-1,0}
                    for (int r = 0; r < W; ++r) cRL[r * W + yc] = endv[r][lane];
            }
            if (k == 0) {
                wL[(size_t)e * N + c] = q;
                if (lc == L - 1)  // G_{0,L-1}
                    for (int r = 0; r < W; ++r) cLR[r * W + yc] = endv[r][lane];
            }
        }
    }
}

template <int W>
static hipError_t launch_refine_w(const mcnegf_kernel& k, const double* onsite,
                                  const double2* G0, float2* Y, int64_t ld, hipStream_t s) {
    MCNEGF_TIMED("refine_kernel", s);
    hipLaunchKernelGGL(refine_kernel<W>, dim3((k.N + 63) / 64, k.nE), dim3(64), 0, s,
                       reinterpret_cast<const double2*>(k.gL), G0, Y, ld, k.energies, onsite,
                       k.gamma, reinterpret_cast<const double2*>(k.sigma), k.gam_lead, k.L, k.t,
                       k.P, k.p_pitch, k.wL, k.wR, reinterpret_cast<double2*>(k.corner),
                       reinterpret_cast<double2*>(k.Gd), k.Adiag);
    return hipGetLastError();
}

hipError_t launch_refine(const mcnegf_kernel& k, const double* onsite, const double2* G0,
                         float2* Y, int64_t ld, hipStream_t s) {
    if (k.W == 16) return launch_refine_w<16>(k, onsite, G0, Y, ld, s);
    if (k.W == 32) return launch_refine_w<32>(k, onsite, G0, Y, ld, s);
    return hipErrorInvalidValue;
}

}  // namespace mcnegf
