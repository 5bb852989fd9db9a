// Shared device helpers and launcher declarations of the mcnegf HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcnegf.h"

namespace mcnegf {

constexpr int kMaxW = 32;
constexpr int kMaxGradW = 32;  // the gradient kernels keep W-vectors in registers
// Outcomes per row (N + 2): the alias build holds 10 bytes per outcome of its row in LDS
// (160 KB per CU), and a packed alias entry has a 16-bit outcome index.
constexpr int kMaxOut = 16320;
constexpr int kMaxGradOut = 16384;  // the back substitution keeps a row in registers
// Packed alias entry: the high 16 bits of the 32-bit threshold over the 16-bit alias; the
// low 16 threshold bits sit in a separate u16 array.
constexpr uint32_t kAliasIdxBits = 16;
constexpr uint32_t kAliasIdxMask = 0xFFFFu;

// ---- complex FP64 arithmetic on double2 (x = real, y = imaginary) ----------------------
__host__ __device__ inline double2 cmk(double re, double im) { return make_double2(re, im); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return cmk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return cmk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
    return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cscale(double2 a, double s) { return cmk(a.x * s, a.y * s); }
__host__ __device__ inline double2 cconj(double2 a) { return cmk(a.x, -a.y); }
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
// a += b * c
__host__ __device__ inline void cfma(double2& a, double2 b, double2 c) {
    a.x = fma(b.x, c.x, fma(-b.y, c.y, a.x));
    a.y = fma(b.x, c.y, fma(b.y, c.x, a.y));
}
// a -= b * c
__host__ __device__ inline void cfms(double2& a, double2 b, double2 c) {
    a.x = fma(-b.x, c.x, fma(b.y, c.y, a.x));
    a.y = fma(-b.x, c.y, fma(-b.y, c.x, a.y));
}
// 1 / a, scaled to avoid overflow
__host__ __device__ inline double2 crecip(double2 a) {
    if (fabs(a.x) >= fabs(a.y)) {
        double r = a.y / a.x, d = a.x + a.y * r;
        return cmk(1.0 / d, -r / d);
    }
    double r = a.x / a.y, d = a.y + a.x * r;
    return cmk(r / d, -1.0 / d);
}
__host__ __device__ inline double2 cdiv(double2 a, double2 b) { return cmul(a, crecip(b)); }

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Position of energy E among the built energies nodes[0 .. nE-1] (ascending) for interpolated
// walks (Sec. V A, "Interpolation"): lo = the last node at or below E, alpha = (E - E_lo) /
// (E_hi - E_lo) as a 32-bit threshold a32 = min(floor(alpha 2^32), 2^32 - 1); at the last node
// lo = nE - 1 and a32 = 0.  An energy outside the nodes, or nodes that do not ascend, set bad
// (the energy is then clamped to the nearest end).
__device__ inline void interp_bracket(const double* nodes, uint32_t nE, double E, uint32_t& lo,
                                      uint32_t& a32, bool& bad) {
    const double first = nodes[0], last = nodes[nE - 1];
    bad = false;
    a32 = 0u;
    if (nE == 1 || !(E > first)) {
        lo = 0;
        bad = !(E == first);
        return;
    }
    if (!(E < last)) {
        lo = nE - 1;
        bad = !(E == last);
        return;
    }
    uint32_t l = 0, h = nE - 1;  // nodes[l] <= E < nodes[h]
    while (h - l > 1) {
        const uint32_t m = (l + h) >> 1;
        if (nodes[m] <= E) l = m; else h = m;
    }
    const double lo_E = nodes[l], hi_E = nodes[l + 1];
    bad = !(hi_E > lo_E);
    const double x = (E - lo_E) / (hi_E - lo_E) * 4294967296.0;
    a32 = x >= 4294967295.0 ? 0xFFFFFFFFu : (x > 0.0 ? (uint32_t)x : 0u);
    lo = l;
}

// The handle restricted to energies [e0, e0 + n): every per-energy array starts at energy e0
// (the status word, counters and reduction scratch are shared).
inline mcnegf_kernel energy_slice(const mcnegf_kernel& k, int e0, int n) {
    mcnegf_kernel c = k;
    const size_t N = k.N, WW = (size_t)k.W * k.W, e = (size_t)e0;
    c.nE = n;
    c.energies = k.energies + e;
    if (k.alias) c.alias = k.alias + e * k.n_out * k.alias_pitch;
    if (k.alias_lo) c.alias_lo = k.alias_lo + e * k.n_out * k.alias_pitch;
    c.P = k.P + e * N * k.p_pitch;
    c.wL = k.wL + e * N;
    c.wR = k.wR + e * N;
    c.Adiag = k.Adiag + e * N;
    c.lead = k.lead + e * MCNEGF_LEAD_NTERMS;
    c.sigma = k.sigma + e * 2 * WW;
    c.gam_lead = k.gam_lead + e * WW;
    c.gL = k.gL + e * 2 * k.L * WW;
    c.gR = k.gR + e * 2 * k.L * WW;
    c.Gd = k.Gd + e * 2 * k.L * WW;
    c.corner = k.corner + e * 4 * WW;
    if (k.direct) c.direct = k.direct + e * (k.p_pitch + 2) * k.p_pitch;
    if (k.direct_vec) c.direct_vec = k.direct_vec + e * 4 * N;
    return c;
}

// ---- workspace layout ------------------------------------------------------------------
struct Layout {
    int64_t alias_pitch, p_pitch;
    uint64_t off_status, off_counters, off_reduce, off_lead, off_sigma, off_gam, off_gL, off_gR,
        off_Gd, off_corner, off_wL, off_wR, off_Adiag, off_P, off_alias, off_alias_lo, off_direct,
        off_direct_vec, off_refine, total;
    int refine_chunk;  // energies refined at a time (FP32 products with one refinement step)
};
Layout make_layout(int W, int L, int nE, bool with_alias, bool with_direct, bool refine = false);
constexpr int kRefineChunk = 8;  // energies refined at a time

// gradient workspace (caller-owned, separate from the build workspace)
struct GradBuffers {
    double2* G;       // [chunk][N][ld] complex G, row-major
    double2* Y;       // [chunk][N][ldY] adjoint solves, column c: Q (c < N) or R (c = N + b)
    double2* part_k;  // [chunk][2][N] dense and diagonal parts of K per site
    double* part_p;   // [chunk][2][N] (P v)_i, (P u)_i
    double* xl;       // [chunk][2][ld] x, lambda
    double* gV;       // [nE][N] dT/dV per energy
    double* gG;       // [nE][N] dT/dgamma per energy
    double* T;        // [nE] DIRECT transmissions (scratch)
    double* sig;      // [nE] (zero)
    int64_t ld, ldY;
};
// Workspace of mc_negf_grad (and mc_negf_grad_mc) with the G-sized buffers for `chunk`
// energies at a time.
uint64_t grad_layout(const mcnegf_kernel& k, int chunk, void* base, GradBuffers* out);

// ---- opt-in launch timing: events around every launch while a profile is attached ------
struct LaunchTimer {
    LaunchTimer(const char* name, hipStream_t s);
    ~LaunchTimer();
    mcnegf_profile* p;
    int slot;
    hipStream_t s;
};
#define MCNEGF_TIMED(name, stream) ::mcnegf::LaunchTimer mcnegf_timer_(name, stream)

// ---- launchers (each defined next to its kernel) ----------------------------------------
hipError_t launch_clear_status(uint32_t* status, uint32_t* counters, hipStream_t s);
hipError_t launch_lead_sigma(const mcnegf_kernel& k, double gamma_l, double delta,
                             hipStream_t s);
hipError_t launch_rgf(const mcnegf_kernel& k, const double* onsite, hipStream_t s);
hipError_t launch_fullinv(const mcnegf_kernel& k, hipStream_t s);
hipError_t launch_fullinv_fp32(const mcnegf_kernel& k, hipStream_t s);
hipError_t launch_fullinv_store_g(const mcnegf_kernel& k, double2* Gc, int64_t ldG,
                                  hipStream_t s);
hipError_t launch_lead_terms(const mcnegf_kernel& k, hipStream_t s);
// rowsum_tol: relative tolerance of the check of each row's total against its spectral value
hipError_t launch_alias_build(const mcnegf_kernel& k, double rowsum_tol, hipStream_t s);
// Transition counts of the walks that reach the collecting lead ([nE][n][n] uint32,
// outcome-major), and the score-function gradient of the Monte Carlo estimator from them.
// Inelastic walks (step 7'): at most kMaxLines energy lines; the walker keeps an exit-energy
// histogram of 2 nE counters in LDS, so nE <= kMaxInelasticE.
constexpr int kMaxLines = 8;
constexpr int kMaxInelasticE = 4096;
hipError_t launch_energy_table(const mcnegf_kernel& k, int n_lines, const int32_t* off,
                               const double* lam, uint64_t* table, hipStream_t s);
hipError_t launch_walk_inelastic(const mcnegf_kernel& k, int n_lines, const int32_t* off,
                                 const uint64_t* table, uint64_t seed, uint32_t tag,
                                 uint32_t walker_begin, uint32_t n_walkers, uint32_t max_steps,
                                 int64_t* tallies, int64_t* hist, hipStream_t s);
hipError_t launch_spectrum(const mcnegf_kernel& k, uint32_t inject_lead, const int64_t* tallies,
                           const int64_t* hist, const double* weights, double* spectrum,
                           hipStream_t s);
hipError_t launch_walk_counts(const mcnegf_kernel& k, uint64_t seed, uint32_t tag,
                              uint32_t walker_begin, uint32_t n_walkers, uint32_t max_steps,
                              uint32_t* counts, int64_t* tallies, hipStream_t s);
hipError_t launch_score_grad(const mcnegf_kernel& k, const GradBuffers& gb,
                             const uint32_t* counts, const int64_t* tallies,
                             uint32_t inject_lead, const double* weights, double* dI_dV,
                             double* dI_dgamma, int chunk, hipStream_t s);
hipError_t launch_grad_reduce(const GradBuffers& gb, const double* weights, int nE, int N,
                              double* dI_dV, double* dI_dgamma, hipStream_t s);
// Importance-sampled walks: alias tables of the modified rows K_ij b_j into the caller's
// tables and rho (per row: modified total / unmodified total); the walks; their estimator.
hipError_t launch_alias_bias(const mcnegf_kernel& k, const double* bias, uint32_t* tables,
                             uint16_t* lows, double* rho, hipStream_t s);
uint64_t weighted_scratch_bytes(int nE, uint64_t n_walkers);
hipError_t launch_walk_weighted(const mcnegf_kernel& k, const uint32_t* tables,
                                const uint16_t* lows, const double* rho, const double* bias,
                                uint64_t seed, uint32_t tag, uint32_t walker_begin,
                                uint32_t n_walkers, uint32_t max_steps, int64_t* tallies,
                                double* wsum, double* partial, hipStream_t s);
hipError_t launch_weighted_current(const mcnegf_kernel& k, uint32_t inject_lead,
                                   const int64_t* tallies, const double* wsum,
                                   const double* weights, double* T, double* sigmaT,
                                   hipStream_t s);
hipError_t launch_walk(const mcnegf_kernel& k, uint64_t seed, uint32_t tag,
                       uint32_t walker_begin, uint32_t n_walkers, uint32_t max_steps,
                       int64_t* tallies, hipStream_t s);
hipError_t launch_mc_current(const mcnegf_kernel& k, uint32_t inject_lead,
                             const int64_t* tallies, const double* weights, double* T,
                             double* sigmaT, hipStream_t s);
hipError_t launch_direct_current(const mcnegf_kernel& k, uint32_t inject_lead,
                                 const double* weights, double* T, double* sigmaT,
                                 hipStream_t s);
hipError_t launch_walk_batch(const mcnegf_batch& b, uint64_t seed, uint32_t walker_begin,
                             uint32_t n_walkers, uint32_t max_steps, const mcnegf_walk_config& c,
                             int64_t* tally_override, hipStream_t s);
hipError_t launch_current_out(const mcnegf_kernel& k, double* d_I_sigma, hipStream_t s);
size_t walk_unit_bytes();
void fill_walk_unit(void* dst, const mcnegf_kernel& k, int e, uint32_t tag, int64_t* tally);
void fill_walk_unit_ids(void* dst, const mcnegf_kernel& k, int e, uint32_t tag, int64_t* tally,
                        const uint32_t* ids, uint32_t nw);
hipError_t launch_walk_units(const void* d_units, uint32_t n_units, const uint32_t* d_chunk_start,
                             uint32_t total_chunks, uint32_t chunk, uint64_t seed,
                             uint32_t max_steps, hipStream_t s);
// scratch of an energy-sampled walk (caller-owned device memory)
struct SampledScratch {
    double* cdf;            // [nE + 1]
    uint32_t* blockhist;    // [nE][blocks]
    uint32_t* blockoff;     // [nE][blocks]
    uint32_t* counts;       // [nE]
    uint32_t* base;         // [nE + 1]
    uint32_t* chunk_start;  // [nE + 1]
    void* units;            // [nE] walk unit descriptors
    uint32_t* draws;        // [n] energy of each walker
    uint32_t* ids;          // [n] walker indices sorted by energy
};
uint64_t sampled_scratch_layout(int nE, uint64_t n, SampledScratch* out, void* base);
// Device address of the library's fixed scratch array (MCNEGF_STATIC_SCRATCH_BYTES) on the
// current device, looked up once per device.
hipError_t static_scratch_address(void** out);
hipError_t launch_walk_sampled(const mcnegf_kernel& k, const SampledScratch& sc, uint64_t seed,
                               uint32_t tag, uint32_t walker_begin, uint32_t n_walkers,
                               uint32_t max_steps, const double* weights, int64_t* tallies,
                               hipStream_t s);
hipError_t launch_sampled_current(const mcnegf_kernel& k, uint32_t inject_lead,
                                  const int64_t* tallies, const double* weights, double* T,
                                  double* sigmaT, hipStream_t s);
// RGF sweeps in FP32 (W = 16 or 32) and the FP64 diagonal blocks, for FP32-products builds.
hipError_t launch_rgf_fp32(const mcnegf_kernel& k, const double* onsite, hipStream_t s);
// The full inverse with FP32 block products, writing the complex G (row-major, pitch ldG).
hipError_t launch_fullinv_fp32_store_g(const mcnegf_kernel& k, double2* Gc, int64_t ldG,
                                       hipStream_t s);
// One FP64 refinement step on the stored G0 (Y: FP32 scratch of the same shape), writing
// |G|^2, the exit weights and the corners of k.
hipError_t launch_refine(const mcnegf_kernel& k, const double* onsite, const double2* G0,
                         float2* Y, int64_t ld, hipStream_t s);
hipError_t launch_walk_interp(const mcnegf_kernel& k, const double* fine, uint32_t nF,
                              uint64_t seed, uint32_t tag, uint32_t walker_begin,
                              uint32_t n_walkers, uint32_t max_steps, int64_t* tallies,
                              hipStream_t s);
hipError_t launch_interp_current(const mcnegf_kernel& k, const double* fine, uint32_t nF,
                                 uint32_t inject_lead, const int64_t* tallies,
                                 const double* weights, double* T, double* sigmaT,
                                 hipStream_t s);
hipError_t launch_interp_distances(const mcnegf_kernel& k, double* dist, hipStream_t s);
hipError_t launch_grad(const mcnegf_kernel& k, const GradBuffers& gb, uint32_t inject_lead,
                       const double* weights, double* dI_dV, double* dI_dgamma, int chunk,
                       hipStream_t s);

}  // namespace mcnegf
