// Lead self-energies and broadenings (Sec. II A, Eqs. (9)-(11); wide-band model Sec. III A,
// Eq. (78)).
//
// Model 0: a clean semi-infinite lead with the wire's W-site cross-section (hopping t, zero
// onsite, hard wall) attached by -t.  Its cross-section Hamiltonian is diagonal in the sine
// modes chi_m(y) = sqrt(2/(W+1)) sin(pi m (y+1)/(W+1)), eps_m = -2t cos(pi m/(W+1)), so
// Sigma = sum_m s_m chi_m chi_m^T with s_m = t^2 g_m, g_m the surface Green's function of a
// chain with onsite eps_m: s_m solves s^2 - (z - eps_m) s + t^2 = 0 at z = E + i delta t.
// The two roots multiply to t^2; the retarded (decaying) one is the smaller in modulus.  It
// is taken as t^2 / s_big with s_big = ((z - eps_m) +- sqrt((z - eps_m)^2 - 4t^2)) / 2,
// the sign chosen so that the two terms add (no cancellation), so no branch of the complex
// square root has to be selected.
// Model 1: Sigma = -(i/2) Gamma_l I on the end slice.
// Gamma = i (Sigma - Sigma^+) = -2 Im Sigma because Sigma is complex symmetric.
#include "common.h"

namespace mcnegf {

__device__ inline double2 csqrt_principal(double2 z) {
    double r = hypot(z.x, z.y);
    if (r == 0.0) return cmk(0.0, 0.0);
    if (z.x >= 0.0) {
        double u = sqrt(0.5 * (r + z.x));
        return cmk(u, z.y / (2.0 * u));
    }
    double v = sqrt(0.5 * (r - z.x));
    if (z.y < 0.0) v = -v;
    return cmk(z.y / (2.0 * v), v);
}

__global__ void __launch_bounds__(256) lead_sigma_kernel(const double* __restrict__ energies,
                                                         int W, double t, int lead_model,
                                                         double gamma_l, double delta,
                                                         double2* __restrict__ sigma,
                                                         double* __restrict__ gam) {
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    __shared__ double2 s_mode[kMaxW];
    __shared__ double chi[kMaxW][kMaxW];
    const double E = energies[e];
    double2* sig = sigma + (size_t)e * W * W;
    double* gm = gam + (size_t)e * W * W;
    if (lead_model == 1) {
        for (int i = tid; i < W * W; i += blockDim.x) {
            const int a = i / W, b = i % W;
            sig[i] = cmk(0.0, a == b ? -0.5 * gamma_l : 0.0);
            gm[i] = a == b ? gamma_l : 0.0;
        }
        return;
    }
    if (tid < W) {
        const int m = tid + 1;
        const double eps = -2.0 * t * cospi((double)m / (double)(W + 1));
        const double2 zm = cmk(E - eps, delta * t);
        const double2 disc = csub(cmul(zm, zm), cmk(4.0 * t * t, 0.0));
        const double2 sq = csqrt_principal(disc);
        const bool plus = (zm.x * sq.x + zm.y * sq.y) >= 0.0;
        const double2 big = cscale(plus ? cadd(zm, sq) : csub(zm, sq), 0.5);
        s_mode[tid] = cscale(crecip(big), t * t);
    }
    for (int i = tid; i < W * W; i += blockDim.x) {
        const int y = i / W, m = i % W;
        chi[y][m] = sqrt(2.0 / (W + 1)) * sinpi((double)((m + 1) * (y + 1)) / (double)(W + 1));
    }
    __syncthreads();
    for (int i = tid; i < W * W; i += blockDim.x) {
        const int a = i / W, b = i % W;
        double2 acc = cmk(0.0, 0.0);
        for (int m = 0; m < W; ++m) acc = cadd(acc, cscale(s_mode[m], chi[a][m] * chi[b][m]));
        sig[i] = acc;
        gm[i] = -2.0 * acc.y;
    }
}

__global__ void clear_status_kernel(uint32_t* status, uint32_t* counters) {
    const int tid = threadIdx.x;
    if (tid == 0) status[0] = 0u;
    if (tid < 64) counters[tid] = 0u;
}

hipError_t launch_clear_status(uint32_t* status, uint32_t* counters, hipStream_t s) {
    {
        MCNEGF_TIMED("clear_status_kernel", s);
        hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(64), 0, s, status, counters);
    }
    return hipGetLastError();
}

hipError_t launch_lead_sigma(const mcnegf_kernel& k, double gamma_l, double delta,
                             hipStream_t s) {
    {
        MCNEGF_TIMED("lead_sigma_kernel", s);
        hipLaunchKernelGGL(lead_sigma_kernel, dim3(k.nE), dim3(256), 0, s, k.energies, k.W, k.t,
                           k.lead_model, gamma_l, delta, reinterpret_cast<double2*>(k.sigma),
                           k.gam_lead);
    }
    return hipGetLastError();
}

}  // namespace mcnegf
