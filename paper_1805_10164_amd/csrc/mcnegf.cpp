// Host side of the C ABI declared in include/mcnegf.h: argument validation, workspace
// layout and the order of the GPU stages.  Every GPU stage runs on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.h"

namespace mcnegf {

static thread_local int32_t g_last_hip_error = 0;
static thread_local mcnegf_profile* g_profile = nullptr;

// A failed event record is not checked here (timing must not change a launch's result): the
// slot's elapsed time then cannot be read, and mc_negf_profile_end returns MCNEGF_EHIP.
LaunchTimer::LaunchTimer(const char* name, hipStream_t stream) : p(g_profile), slot(-1), s(stream) {
    if (!p) return;
    if (p->n >= MCNEGF_PROFILE_MAX) {
        ++p->dropped;
        return;
    }
    slot = p->n++;
    p->name[slot] = name;
    (void)hipEventRecord(p->start[slot], s);
}

LaunchTimer::~LaunchTimer() {
    if (p && slot >= 0) (void)hipEventRecord(p->stop[slot], s);
}

static int32_t hip_fail(hipError_t e) {
    g_last_hip_error = (int32_t)e;
    return MCNEGF_EHIP;
}

static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

Layout make_layout(int W, int L, int nE, bool with_alias, bool with_direct, bool refine) {
    Layout o;
    const int64_t N = (int64_t)W * L;
    const int64_t n = N + 2;
    o.alias_pitch = round_up(n, 16);
    o.p_pitch = round_up(N, 16);
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = off;
        off = align256(off + bytes);
        return at;
    };
    o.off_status = take(256);
    o.off_counters = take(64 * 4);
    o.off_reduce = take((uint64_t)(nE + 8) * 8);
    o.off_lead = take((uint64_t)nE * MCNEGF_LEAD_NTERMS * 8);
    o.off_sigma = take((uint64_t)nE * W * W * 16);
    o.off_gam = take((uint64_t)nE * W * W * 8);
    o.off_gL = take((uint64_t)nE * L * W * W * 16);
    o.off_gR = take((uint64_t)nE * L * W * W * 16);
    o.off_Gd = take((uint64_t)nE * L * W * W * 16);
    o.off_corner = take((uint64_t)nE * 2 * W * W * 16);
    o.off_wL = take((uint64_t)nE * N * 8);
    o.off_wR = take((uint64_t)nE * N * 8);
    o.off_Adiag = take((uint64_t)nE * N * 8);
    o.off_direct_vec = take(with_direct ? (uint64_t)nE * 4 * N * 8 : 0);
    o.off_P = take((uint64_t)nE * N * o.p_pitch * 8);
    o.off_alias = take(with_alias ? (uint64_t)nE * n * o.alias_pitch * 4 : 0);
    o.off_alias_lo = take(with_alias ? (uint64_t)nE * n * o.alias_pitch * 2 : 0);
    o.off_direct = take(with_direct ? (uint64_t)nE * (o.p_pitch + 2) * o.p_pitch * 8 : 0);
    // refinement scratch: G0 (complex FP64) and the FP32 forward solves, for a chunk of energies
    o.refine_chunk = refine ? (nE < kRefineChunk ? nE : kRefineChunk) : 0;
    o.off_refine = take((uint64_t)o.refine_chunk * N * o.p_pitch * 24);
    o.total = off;
    return o;
}

static bool valid_system(const mcnegf_system* s) {
    if (!s) return false;
    if (s->W < 1 || s->W > kMaxW || s->L < 1) return false;
    if ((int64_t)s->W * s->L + 2 > kMaxOut) return false;
    if (!(s->t > 0.0) || !std::isfinite(s->t)) return false;
    if (s->lead_model == 0) {
        if (!(s->delta_lead > 0.0) || !std::isfinite(s->delta_lead)) return false;
    } else if (s->lead_model == 1) {
        if (!(s->gamma_l >= 0.0) || !std::isfinite(s->gamma_l)) return false;
    } else {
        return false;
    }
    if (s->flags & ~(MCNEGF_BUILD_NO_ALIAS | MCNEGF_BUILD_NO_DIRECT | MCNEGF_BUILD_FP32_PRODUCTS |
                     MCNEGF_BUILD_FP32_REFINE | MCNEGF_BUILD_FP32_SWEEPS))
        return false;
    if ((s->flags & MCNEGF_BUILD_FP32_PRODUCTS) && s->W != 16 && s->W != 32) return false;
    if ((s->flags & (MCNEGF_BUILD_FP32_REFINE | MCNEGF_BUILD_FP32_SWEEPS)) &&
        !(s->flags & MCNEGF_BUILD_FP32_PRODUCTS))
        return false;
    return true;
}

static bool with_alias(const mcnegf_system* s) { return !(s->flags & MCNEGF_BUILD_NO_ALIAS); }
static bool with_direct(const mcnegf_system* s) { return !(s->flags & MCNEGF_BUILD_NO_DIRECT); }
static bool with_refine(const mcnegf_system* s) { return (s->flags & MCNEGF_BUILD_FP32_REFINE) != 0; }
static Layout layout_of(const mcnegf_system* s, int nE) {
    return make_layout(s->W, s->L, nE, with_alias(s), with_direct(s), with_refine(s));
}

// A handle as mc_negf_build_kernel fills it: sizes consistent (compared in 64 bits, so a
// corrupt handle cannot overflow them), rows within the 16-bit alias indices, buffers set.
static bool valid_kernel(const mcnegf_kernel* k) {
    return k && k->W >= 1 && k->W <= kMaxW && k->L >= 1 &&
           (int64_t)k->N == (int64_t)k->W * k->L && (int64_t)k->n_out == (int64_t)k->N + 2 &&
           k->n_out <= kMaxOut && k->nE >= 1 && k->p_pitch >= k->N && k->p_pitch % 16 == 0 &&
           k->P && k->lead && k->status && k->counters && k->reduce;
}

static int32_t status_to_code(uint32_t flags, bool mc) {
    if (flags & (MCNEGF_FLAG_NONFINITE | MCNEGF_FLAG_SINGULAR | MCNEGF_FLAG_NOTSPD))
        return MCNEGF_ENUMERIC;
    if (mc && (flags & MCNEGF_FLAG_TRUNC)) return MCNEGF_WTRUNC;
    if (flags & MCNEGF_FLAG_ROWSUM) return MCNEGF_WNUMERIC;
    return MCNEGF_OK;
}

uint64_t grad_layout(const mcnegf_kernel& k, int chunk, void* base, GradBuffers* out) {
    const int64_t N = k.N, nE = k.nE, ld = k.p_pitch, ldY = round_up(N + 2 * k.W, 16);
    const int64_t nc = chunk;
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = off;
        off = align256(off + bytes);
        return at;
    };
    const uint64_t oG = take((uint64_t)nc * N * ld * 16);
    const uint64_t oY = take((uint64_t)nc * N * ldY * 16);
    const uint64_t oK = take((uint64_t)nc * 2 * N * 16);
    const uint64_t oP = take((uint64_t)nc * 2 * N * 8);
    const uint64_t oX = take((uint64_t)nc * 2 * ld * 8);
    const uint64_t oV = take((uint64_t)nE * N * 8);
    const uint64_t oGg = take((uint64_t)nE * N * 8);
    const uint64_t oT = take((uint64_t)nE * 8);
    const uint64_t oS = take((uint64_t)nE * 8);
    if (out) {
        char* b = static_cast<char*>(base);
        out->G = reinterpret_cast<double2*>(b + oG);
        out->Y = reinterpret_cast<double2*>(b + oY);
        out->part_k = reinterpret_cast<double2*>(b + oK);
        out->part_p = reinterpret_cast<double*>(b + oP);
        out->xl = reinterpret_cast<double*>(b + oX);
        out->gV = reinterpret_cast<double*>(b + oV);
        out->gG = reinterpret_cast<double*>(b + oGg);
        out->T = reinterpret_cast<double*>(b + oT);
        out->sig = reinterpret_cast<double*>(b + oS);
        out->ld = ld;
        out->ldY = ldY;
    }
    return off;
}

}  // namespace mcnegf

using namespace mcnegf;

extern "C" {

int32_t mc_negf_version(void) { return 10000; }

int32_t mc_negf_last_hip_error(void) { return g_last_hip_error; }

int32_t mc_negf_workspace_bytes(const mcnegf_system* sys, int32_t nE, uint64_t* bytes_out) {
    if (!valid_system(sys) || nE < 1 || !bytes_out) return MCNEGF_EINVAL;
    *bytes_out = layout_of(sys, nE).total;
    return MCNEGF_OK;
}

int32_t mc_negf_build_kernel(const mcnegf_system* sys, const double* d_onsite,
                             const double* d_gamma, const double* d_energies, int32_t nE,
                             void* d_ws, uint64_t ws_bytes, mcnegf_kernel* out,
                             hipStream_t stream) {
    if (!valid_system(sys) || !d_onsite || !d_gamma || !d_energies || nE < 1 || !d_ws || !out)
        return MCNEGF_EINVAL;
    if (((uintptr_t)d_ws & 255u) != 0) return MCNEGF_EINVAL;
    const Layout lay = layout_of(sys, nE);
    if (ws_bytes < lay.total) return MCNEGF_EWS;
    char* base = static_cast<char*>(d_ws);
    mcnegf_kernel k;
    std::memset(&k, 0, sizeof(k));
    k.W = sys->W;
    k.L = sys->L;
    k.N = sys->W * sys->L;
    k.n_out = k.N + 2;
    k.nE = nE;
    k.lead_model = sys->lead_model;
    k.t = sys->t;
    k.delta_lead = sys->lead_model == 0 ? sys->delta_lead : 0.0;
    k.alias_pitch = lay.alias_pitch;
    k.p_pitch = lay.p_pitch;
    k.energies = d_energies;
    k.gamma = d_gamma;
    if (with_alias(sys)) {
        k.alias = reinterpret_cast<uint32_t*>(base + lay.off_alias);
        k.alias_lo = reinterpret_cast<uint16_t*>(base + lay.off_alias_lo);
    }
    k.P = reinterpret_cast<double*>(base + lay.off_P);
    k.wL = reinterpret_cast<double*>(base + lay.off_wL);
    k.wR = reinterpret_cast<double*>(base + lay.off_wR);
    k.Adiag = reinterpret_cast<double*>(base + lay.off_Adiag);
    k.lead = reinterpret_cast<double*>(base + lay.off_lead);
    k.sigma = reinterpret_cast<double*>(base + lay.off_sigma);
    k.gam_lead = reinterpret_cast<double*>(base + lay.off_gam);
    k.gL = reinterpret_cast<double*>(base + lay.off_gL);
    k.gR = reinterpret_cast<double*>(base + lay.off_gR);
    k.Gd = reinterpret_cast<double*>(base + lay.off_Gd);
    k.corner = reinterpret_cast<double*>(base + lay.off_corner);
    if (with_direct(sys)) {
        k.direct = reinterpret_cast<double*>(base + lay.off_direct);
        k.direct_vec = reinterpret_cast<double*>(base + lay.off_direct_vec);
    }
    k.reduce = reinterpret_cast<double*>(base + lay.off_reduce);
    k.status = reinterpret_cast<uint32_t*>(base + lay.off_status);
    k.counters = reinterpret_cast<uint32_t*>(base + lay.off_counters);
    k.ws = d_ws;
    k.ws_bytes = ws_bytes;

    hipError_t err;
    if ((err = launch_clear_status(k.status, k.counters, stream)) != hipSuccess) return hip_fail(err);
    if ((err = launch_lead_sigma(k, sys->gamma_l, sys->delta_lead, stream)) != hipSuccess)
        return hip_fail(err);
    if ((err = (sys->flags & MCNEGF_BUILD_FP32_SWEEPS) ? launch_rgf_fp32(k, d_onsite, stream)
                                                            : launch_rgf(k, d_onsite, stream)) !=
        hipSuccess)
        return hip_fail(err);
    if (with_refine(sys)) {
        // FP32 block products, then one FP64 refinement step, a chunk of energies at a time
        double2* G0 = reinterpret_cast<double2*>(base + lay.off_refine);
        float2* Y = reinterpret_cast<float2*>(base + lay.off_refine +
                                              (uint64_t)lay.refine_chunk * k.N * k.p_pitch * 16);
        for (int e0 = 0; e0 < nE; e0 += lay.refine_chunk) {
            const mcnegf_kernel kc = energy_slice(k, e0, std::min(lay.refine_chunk, nE - e0));
            if ((err = launch_fullinv_fp32_store_g(kc, G0, k.p_pitch, stream)) != hipSuccess)
                return hip_fail(err);
            if ((err = launch_refine(kc, d_onsite, G0, Y, k.p_pitch, stream)) != hipSuccess)
                return hip_fail(err);
        }
    } else if ((err = (sys->flags & MCNEGF_BUILD_FP32_PRODUCTS) ? launch_fullinv_fp32(k, stream)
                                                                   : launch_fullinv(k, stream)) !=
               hipSuccess) {
        return hip_fail(err);
    }
    if ((err = launch_lead_terms(k, stream)) != hipSuccess) return hip_fail(err);
    // row totals against A_jj and Tr Gamma_p A: FP64 products (and refined FP32 products)
    // agree to rounding, FP32 block products to their own rounding accumulated over the slices
    const double rowsum_tol =
        (sys->flags & MCNEGF_BUILD_FP32_PRODUCTS) && !with_refine(sys) ? 1e-4 : 1e-8;
    if (with_alias(sys) && (err = launch_alias_build(k, rowsum_tol, stream)) != hipSuccess)
        return hip_fail(err);
    *out = k;
    return MCNEGF_OK;
}

int32_t mc_negf_walk(const mcnegf_kernel* k, uint64_t seed, uint32_t realization,
                     uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers_per_energy,
                     uint32_t max_steps, int64_t* d_tallies, hipStream_t stream) {
    if (!valid_kernel(k) || !k->alias || !k->alias_lo || !d_tallies || inject_lead > 1 ||
        realization >= (1u << 30) || max_steps < 1)
        return MCNEGF_EINVAL;
    // walker indices and the end of the range are held in 32 bits
    if (walker_begin >= 0x100000000ull || n_walkers_per_energy >= 0x100000000ull ||
        walker_begin + n_walkers_per_energy >= 0x100000000ull)
        return MCNEGF_EINVAL;
    if (n_walkers_per_energy == 0) return MCNEGF_OK;
    const uint32_t tag = (realization << 1) | inject_lead;
    hipError_t err = launch_walk(*k, seed, tag, (uint32_t)walker_begin,
                                 (uint32_t)n_walkers_per_energy, max_steps, d_tallies, stream);
    if (err != hipSuccess) return hip_fail(err);
    return MCNEGF_OK;
}

int32_t mc_negf_current(const mcnegf_kernel* k, int32_t mode, uint32_t inject_lead,
                        const int64_t* d_tallies, const double* d_weights, double* d_T,
                        double* d_sigmaT, double* h_I_sigma, hipStream_t stream) {
    if (!valid_kernel(k) || !d_weights || !d_T || !d_sigmaT || !h_I_sigma || inject_lead > 1)
        return MCNEGF_EINVAL;
    hipError_t err;
    if (mode == 0 || mode == 2) {
        if (!d_tallies || !k->alias) return MCNEGF_EINVAL;  // tallies need a walked kernel
        err = mode == 0 ? launch_mc_current(*k, inject_lead, d_tallies, d_weights, d_T, d_sigmaT,
                                            stream)
                        : launch_sampled_current(*k, inject_lead, d_tallies, d_weights, d_T,
                                                 d_sigmaT, stream);
    } else if (mode == 1) {
        if (!k->direct || !k->direct_vec) return MCNEGF_EINVAL;
        err = launch_direct_current(*k, inject_lead, d_weights, d_T, d_sigmaT, stream);
    } else {
        return MCNEGF_EINVAL;
    }
    if (err != hipSuccess) return hip_fail(err);
    double host[2];
    uint32_t flags = 0;
    if ((err = hipMemcpyAsync(host, k->reduce, sizeof(host), hipMemcpyDeviceToHost, stream)) !=
        hipSuccess)
        return hip_fail(err);
    if ((err = hipMemcpyAsync(&flags, k->status, sizeof(flags), hipMemcpyDeviceToHost, stream)) !=
        hipSuccess)
        return hip_fail(err);
    if ((err = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(err);
    h_I_sigma[0] = host[0];
    h_I_sigma[1] = std::sqrt(host[1] > 0.0 ? host[1] : 0.0);
    return status_to_code(flags, mode != 1);
}

int32_t mc_negf_grad_workspace_bytes(const mcnegf_kernel* k, uint64_t* bytes_out) {
    if (!valid_kernel(k) || !bytes_out) return MCNEGF_EINVAL;
    *bytes_out = grad_layout(*k, k->nE, nullptr, nullptr);
    return MCNEGF_OK;
}

int32_t mc_negf_grad_workspace_bytes_chunk(const mcnegf_kernel* k, int32_t chunk,
                                           uint64_t* bytes_out) {
    if (!valid_kernel(k) || !bytes_out || chunk < 1 || chunk > k->nE) return MCNEGF_EINVAL;
    *bytes_out = grad_layout(*k, chunk, nullptr, nullptr);
    return MCNEGF_OK;
}

int32_t mc_negf_grad(const mcnegf_kernel* k, uint32_t inject_lead, const double* d_weights,
                     void* d_gws, uint64_t gws_bytes, double* d_dI_dV, double* d_dI_dgamma,
                     double* h_I, hipStream_t stream) {
    if (!valid_kernel(k) || !d_weights || !d_gws || !d_dI_dV || !d_dI_dgamma || !h_I ||
        inject_lead > 1 || !k->direct || !k->direct_vec || k->W > kMaxGradW ||
        k->p_pitch > kMaxGradOut)
        return MCNEGF_EINVAL;
    // the largest chunk of energies whose G-sized buffers fit the workspace
    if (grad_layout(*k, 1, nullptr, nullptr) > gws_bytes) return MCNEGF_EWS;
    int lo = 1, hi = k->nE;
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        if (grad_layout(*k, mid, nullptr, nullptr) <= gws_bytes) lo = mid; else hi = mid - 1;
    }
    const int chunk = lo;
    GradBuffers gb;
    grad_layout(*k, chunk, d_gws, &gb);
    hipError_t err = launch_direct_current(*k, inject_lead, d_weights, gb.T, gb.sig, stream);
    if (err != hipSuccess) return hip_fail(err);
    if ((err = launch_grad(*k, gb, inject_lead, d_weights, d_dI_dV, d_dI_dgamma, chunk, stream)) !=
        hipSuccess)
        return hip_fail(err);
    double host[2];
    uint32_t flags = 0;
    if ((err = hipMemcpyAsync(host, k->reduce, sizeof(host), hipMemcpyDeviceToHost, stream)) !=
        hipSuccess)
        return hip_fail(err);
    if ((err = hipMemcpyAsync(&flags, k->status, sizeof(flags), hipMemcpyDeviceToHost, stream)) !=
        hipSuccess)
        return hip_fail(err);
    if ((err = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(err);
    *h_I = host[0];
    return status_to_code(flags, false);
}

// ---- score-function gradient of the Monte Carlo estimator ------------------------------

int32_t mc_negf_walk_counts_bytes(const mcnegf_kernel* k, uint64_t* bytes_out) {
    if (!valid_kernel(k) || !bytes_out) return MCNEGF_EINVAL;
    *bytes_out = (uint64_t)k->nE * (uint64_t)k->n_out * (uint64_t)k->n_out * 4;
    return MCNEGF_OK;
}

int32_t mc_negf_walk_counts(const mcnegf_kernel* k, uint64_t seed, uint32_t realization,
                            uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers,
                            uint32_t max_steps, uint32_t* d_counts, int64_t* d_tallies,
                            hipStream_t stream) {
    if (!valid_kernel(k) || !k->alias || !k->alias_lo || !d_counts || !d_tallies ||
        inject_lead > 1 || realization >= (1u << 30) || max_steps < 1)
        return MCNEGF_EINVAL;
    if (walker_begin >= 0x100000000ull || n_walkers >= 0x100000000ull ||
        walker_begin + n_walkers >= 0x100000000ull)
        return MCNEGF_EINVAL;
    const uint32_t tag = (realization << 1) | inject_lead;
    hipError_t err = launch_walk_counts(*k, seed, tag, (uint32_t)walker_begin,
                                        (uint32_t)n_walkers, max_steps, d_counts, d_tallies,
                                        stream);
    return err == hipSuccess ? MCNEGF_OK : hip_fail(err);
}

int32_t mc_negf_grad_mc(const mcnegf_kernel* k, uint32_t inject_lead, const uint32_t* d_counts,
                        const int64_t* d_tallies, const double* d_weights, void* d_gws,
                        uint64_t gws_bytes, double* d_dI_dV, double* d_dI_dgamma,
                        hipStream_t stream) {
    if (!valid_kernel(k) || !d_counts || !d_tallies || !d_weights || !d_gws || !d_dI_dV ||
        !d_dI_dgamma || inject_lead > 1 || k->W > kMaxGradW || !k->wL || !k->wR ||
        !k->Adiag || !k->gam_lead || !k->corner || !k->gamma)
        return MCNEGF_EINVAL;
    if (grad_layout(*k, 1, nullptr, nullptr) > gws_bytes) return MCNEGF_EWS;
    int lo = 1, hi = k->nE;
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        if (grad_layout(*k, mid, nullptr, nullptr) <= gws_bytes) lo = mid; else hi = mid - 1;
    }
    GradBuffers gb;
    grad_layout(*k, lo, d_gws, &gb);
    hipError_t err = launch_score_grad(*k, gb, d_counts, d_tallies, inject_lead, d_weights,
                                       d_dI_dV, d_dI_dgamma, lo, stream);
    return err == hipSuccess ? MCNEGF_OK : hip_fail(err);
}

// ---- inelastic walks (step 7') -----------------------------------------------------------

// Host check of the energy lines: 1..kMaxLines lines, |offset| < nE, lambda finite and >= 0,
// and from every energy some line of positive weight stays on the grid.
static bool valid_lines(const mcnegf_kernel& k, int32_t n_lines, const int32_t* off,
                        const double* lam) {
    if (n_lines < 1 || n_lines > kMaxLines || !off) return false;
    for (int j = 0; j < n_lines; ++j)
        if (off[j] <= -k.nE || off[j] >= k.nE) return false;
    if (lam) {
        for (int j = 0; j < n_lines; ++j)
            if (!(lam[j] >= 0.0) || !std::isfinite(lam[j])) return false;
        for (int e = 0; e < k.nE; ++e) {
            bool any = false;
            for (int j = 0; j < n_lines; ++j)
                any = any || (lam[j] > 0.0 && e + off[j] >= 0 && e + off[j] < k.nE);
            if (!any) return false;
        }
    }
    return true;
}

int32_t mc_negf_energy_table_bytes(const mcnegf_kernel* k, int32_t n_lines,
                                   uint64_t* bytes_out) {
    if (!valid_kernel(k) || !bytes_out || n_lines < 1 || n_lines > kMaxLines)
        return MCNEGF_EINVAL;
    *bytes_out = (uint64_t)k->nE * (uint64_t)k->N * (uint64_t)n_lines * 8;
    return MCNEGF_OK;
}

int32_t mc_negf_energy_table(const mcnegf_kernel* k, int32_t n_lines, const int32_t* h_offsets,
                             const double* h_lambda, uint64_t* d_table, uint64_t table_bytes,
                             hipStream_t stream) {
    if (!valid_kernel(k) || !k->Adiag || !d_table || !h_lambda ||
        !valid_lines(*k, n_lines, h_offsets, h_lambda))
        return MCNEGF_EINVAL;
    if (table_bytes < (uint64_t)k->nE * (uint64_t)k->N * (uint64_t)n_lines * 8)
        return MCNEGF_EWS;
    hipError_t err = launch_energy_table(*k, n_lines, h_offsets, h_lambda, d_table, stream);
    return err == hipSuccess ? MCNEGF_OK : hip_fail(err);
}

int32_t mc_negf_walk_inelastic(const mcnegf_kernel* k, int32_t n_lines, const int32_t* h_offsets,
                               const uint64_t* d_table, uint64_t table_bytes, uint64_t seed,
                               uint32_t realization,
                               uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers,
                               uint32_t max_steps, int64_t* d_tallies, int64_t* d_hist,
                               hipStream_t stream) {
    if (!valid_kernel(k) || !k->alias || !k->alias_lo || !d_table || !d_tallies || !d_hist ||
        !valid_lines(*k, n_lines, h_offsets, nullptr) || k->nE > kMaxInelasticE ||
        (uint64_t)k->n_out * (uint64_t)k->alias_pitch >= 0x100000000ull ||
        inject_lead > 1 || realization >= (1u << 30) || max_steps < 1)
        return MCNEGF_EINVAL;
    if (walker_begin >= 0x100000000ull || n_walkers >= 0x100000000ull ||
        walker_begin + n_walkers >= 0x100000000ull)
        return MCNEGF_EINVAL;
    if (table_bytes < (uint64_t)k->nE * (uint64_t)k->N * (uint64_t)n_lines * 8) return MCNEGF_EWS;
    const uint32_t tag = (realization << 1) | inject_lead;
    hipError_t err = launch_walk_inelastic(*k, n_lines, h_offsets, d_table, seed, tag,
                                           (uint32_t)walker_begin, (uint32_t)n_walkers,
                                           max_steps, d_tallies, d_hist, stream);
    return err == hipSuccess ? MCNEGF_OK : hip_fail(err);
}

int32_t mc_negf_spectrum(const mcnegf_kernel* k, uint32_t inject_lead, const int64_t* d_tallies,
                         const int64_t* d_hist, const double* d_weights, double* d_spectrum,
                         hipStream_t stream) {
    if (!valid_kernel(k) || !k->lead || !d_tallies || !d_hist || !d_weights || !d_spectrum ||
        inject_lead > 1)
        return MCNEGF_EINVAL;
    hipError_t err = launch_spectrum(*k, inject_lead, d_tallies, d_hist, d_weights, d_spectrum,
                                     stream);
    return err == hipSuccess ? MCNEGF_OK : hip_fail(err);
}

int32_t mc_negf_profile_begin(mcnegf_profile* p) {
    if (!p || g_profile) return MCNEGF_EINVAL;
    std::memset(p, 0, sizeof(*p));
    for (int i = 0; i < MCNEGF_PROFILE_MAX; ++i) {
        hipError_t err;
        if ((err = hipEventCreate(&p->start[i])) != hipSuccess ||
            (err = hipEventCreate(&p->stop[i])) != hipSuccess) {
            for (int j = 0; j <= i; ++j) {  // cleanup: a failed destroy leaves nothing to do
                if (p->start[j]) (void)hipEventDestroy(p->start[j]);
                if (p->stop[j]) (void)hipEventDestroy(p->stop[j]);
            }
            std::memset(p, 0, sizeof(*p));
            return hip_fail(err);
        }
    }
    g_profile = p;
    return MCNEGF_OK;
}

int32_t mc_negf_profile_end(mcnegf_profile* p, float* ms_out) {
    if (!p || g_profile != p) return MCNEGF_EINVAL;
    g_profile = nullptr;
    int32_t rc = MCNEGF_OK;
    for (int i = 0; i < p->n; ++i) {
        float ms = 0.0f;
        hipError_t err = hipEventSynchronize(p->stop[i]);
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, p->start[i], p->stop[i]);
        if (err != hipSuccess) rc = hip_fail(err);
        if (ms_out) ms_out[i] = ms;
    }
    for (int i = 0; i < MCNEGF_PROFILE_MAX; ++i) {
        (void)hipEventDestroy(p->start[i]);
        (void)hipEventDestroy(p->stop[i]);
    }
    return rc;
}

int32_t mc_negf_status(const mcnegf_kernel* k, uint32_t* h_flags, hipStream_t stream) {
    if (!valid_kernel(k) || !h_flags) return MCNEGF_EINVAL;
    hipError_t err;
    if ((err = hipMemcpyAsync(h_flags, k->status, sizeof(uint32_t), hipMemcpyDeviceToHost,
                              stream)) != hipSuccess)
        return hip_fail(err);
    if ((err = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(err);
    return MCNEGF_OK;
}

int32_t mc_negf_current_async(const mcnegf_kernel* k, int32_t mode, uint32_t inject_lead,
                              const int64_t* d_tallies, const double* d_weights, double* d_T,
                              double* d_sigmaT, double* d_I_sigma, hipStream_t stream) {
    if (!valid_kernel(k) || !d_weights || !d_T || !d_sigmaT || !d_I_sigma || inject_lead > 1)
        return MCNEGF_EINVAL;
    hipError_t err;
    if (mode == 0 || mode == 2) {
        if (!d_tallies || !k->alias) return MCNEGF_EINVAL;
        err = mode == 0 ? launch_mc_current(*k, inject_lead, d_tallies, d_weights, d_T, d_sigmaT,
                                            stream)
                        : launch_sampled_current(*k, inject_lead, d_tallies, d_weights, d_T,
                                                 d_sigmaT, stream);
    } else if (mode == 1) {
        if (!k->direct || !k->direct_vec) return MCNEGF_EINVAL;
        err = launch_direct_current(*k, inject_lead, d_weights, d_T, d_sigmaT, stream);
    } else {
        return MCNEGF_EINVAL;
    }
    if (err != hipSuccess) return hip_fail(err);
    if ((err = launch_current_out(*k, d_I_sigma, stream)) != hipSuccess) return hip_fail(err);
    return MCNEGF_OK;
}

constexpr int kMaxSampledEnergies = 16384;  // one u32 counter per energy in LDS

int32_t mc_negf_walk_sampled_bytes(const mcnegf_kernel* k, uint64_t n_walkers,
                                   uint64_t* bytes_out) {
    if (!valid_kernel(k) || !bytes_out || k->nE > kMaxSampledEnergies ||
        n_walkers > 0xffffffffull)
        return MCNEGF_EINVAL;
    *bytes_out = sampled_scratch_layout(k->nE, n_walkers, nullptr, nullptr);
    return MCNEGF_OK;
}

static bool valid_sampled_args(const mcnegf_kernel* k, uint32_t realization,
                               uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers,
                               uint32_t max_steps, const double* d_weights,
                               const int64_t* d_tallies) {
    if (!valid_kernel(k) || !k->alias || !k->alias_lo || !d_weights || !d_tallies ||
        inject_lead > 1 || realization >= (1u << 30) || max_steps < 1 ||
        k->nE > kMaxSampledEnergies)
        return false;
    return walker_begin < 0x100000000ull && n_walkers < 0x100000000ull &&
           walker_begin + n_walkers < 0x100000000ull;
}

int32_t mc_negf_walk_sampled(const mcnegf_kernel* k, uint64_t seed, uint32_t realization,
                             uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers,
                             uint32_t max_steps, const double* d_weights, int64_t* d_tallies,
                             void* d_scratch, uint64_t scratch_bytes, hipStream_t stream) {
    if (!valid_sampled_args(k, realization, inject_lead, walker_begin, n_walkers, max_steps,
                            d_weights, d_tallies) ||
        !d_scratch)
        return MCNEGF_EINVAL;
    if (((uintptr_t)d_scratch & 255u) != 0) return MCNEGF_EWS;
    SampledScratch sc;
    if (sampled_scratch_layout(k->nE, n_walkers, &sc, d_scratch) > scratch_bytes)
        return MCNEGF_EWS;
    if (n_walkers == 0) return MCNEGF_OK;
    const uint32_t tag = (realization << 1) | inject_lead;
    hipError_t err = launch_walk_sampled(*k, sc, seed, tag, (uint32_t)walker_begin,
                                         (uint32_t)n_walkers, max_steps, d_weights, d_tallies,
                                         stream);
    return err == hipSuccess ? MCNEGF_OK : hip_fail(err);
}

int32_t mc_negf_walk_sampled_noalloc(const mcnegf_kernel* k, uint64_t seed,
                                     uint32_t realization, uint32_t inject_lead,
                                     uint64_t walker_begin, uint64_t n_walkers,
                                     uint32_t max_steps, const double* d_weights,
                                     int64_t* d_tallies, hipStream_t stream) {
    if (!valid_sampled_args(k, realization, inject_lead, walker_begin, n_walkers, max_steps,
                            d_weights, d_tallies))
        return MCNEGF_EINVAL;
    // the fixed scratch must hold the draws, the walker lists and the per-energy tables
    if (sampled_scratch_layout(k->nE, n_walkers, nullptr, nullptr) > MCNEGF_STATIC_SCRATCH_BYTES)
        return MCNEGF_EWS;
    if (n_walkers == 0) return MCNEGF_OK;
    void* base = nullptr;
    hipError_t err = static_scratch_address(&base);
    if (err != hipSuccess) return hip_fail(err);
    SampledScratch sc;
    sampled_scratch_layout(k->nE, n_walkers, &sc, base);
    const uint32_t tag = (realization << 1) | inject_lead;
    err = launch_walk_sampled(*k, sc, seed, tag, (uint32_t)walker_begin, (uint32_t)n_walkers,
                              max_steps, d_weights, d_tallies, stream);
    return err == hipSuccess ? MCNEGF_OK : hip_fail(err);
}

// ---- interpolated step-6' probabilities (Sec. V A, "Interpolation") ---------------------

int32_t mc_negf_interp_distances(const mcnegf_kernel* k, double* d_dist, hipStream_t stream) {
    if (!valid_kernel(k) || !d_dist || k->nE < 2 || !k->wL || !k->wR || !k->gamma)
        return MCNEGF_EINVAL;
    hipError_t err = launch_interp_distances(*k, d_dist, stream);
    return err == hipSuccess ? MCNEGF_OK : hip_fail(err);
}

int32_t mc_negf_interp_plan(const double* h_nodes, int32_t nN, const double* h_dist,
                            const double* h_fine, int32_t nF, double tol, int32_t* h_exact,
                            int32_t* n_exact) {
    if (!h_nodes || nN < 1 || (nN > 1 && !h_dist) || !h_fine || nF < 1 || !h_exact ||
        !n_exact || !(tol >= 0.0))
        return MCNEGF_EINVAL;
    for (int32_t i = 0; i + 1 < nN; ++i)
        if (!(h_nodes[i + 1] > h_nodes[i])) return MCNEGF_EINVAL;
    int32_t m = 0;
    for (int32_t f = 0; f < nF; ++f) {
        const double E = h_fine[f];
        if (!(E >= h_nodes[0]) || !(E <= h_nodes[nN - 1])) return MCNEGF_EINVAL;
        // the interval [nodes[lo], nodes[lo + 1]) holding E; a node itself is exact already
        const int32_t lo = (int32_t)(std::upper_bound(h_nodes, h_nodes + nN, E) - h_nodes) - 1;
        if (E == h_nodes[lo]) continue;
        if (!(h_dist[lo] <= tol)) h_exact[m++] = f;
    }
    *n_exact = m;
    return MCNEGF_OK;
}

static bool valid_interp_walk(const mcnegf_kernel* k, const double* fine, int32_t nF,
                              uint32_t realization, uint32_t inject_lead, uint64_t walker_begin,
                              uint64_t n_walkers, uint32_t max_steps, const int64_t* tallies) {
    if (!valid_kernel(k) || !k->alias || !k->alias_lo || !fine || nF < 1 || nF > 0x7FFFFFFE ||
        !tallies || inject_lead > 1 || realization >= (1u << 30) || max_steps < 1)
        return false;
    return walker_begin < 0x100000000ull && n_walkers < 0x100000000ull &&
           walker_begin + n_walkers < 0x100000000ull;
}

int32_t mc_negf_walk_interp(const mcnegf_kernel* k, const double* d_fine_energies, int32_t nF,
                            uint64_t seed, uint32_t realization, uint32_t inject_lead,
                            uint64_t walker_begin, uint64_t n_walkers_per_energy,
                            uint32_t max_steps, int64_t* d_tallies, hipStream_t stream) {
    if (!valid_interp_walk(k, d_fine_energies, nF, realization, inject_lead, walker_begin,
                           n_walkers_per_energy, max_steps, d_tallies))
        return MCNEGF_EINVAL;
    if (n_walkers_per_energy == 0) return MCNEGF_OK;
    const uint32_t tag = (realization << 1) | inject_lead;
    hipError_t err = launch_walk_interp(*k, d_fine_energies, (uint32_t)nF, seed, tag,
                                        (uint32_t)walker_begin, (uint32_t)n_walkers_per_energy,
                                        max_steps, d_tallies, stream);
    return err == hipSuccess ? MCNEGF_OK : hip_fail(err);
}

int32_t mc_negf_current_interp(const mcnegf_kernel* k, const double* d_fine_energies,
                               int32_t nF, uint32_t inject_lead, const int64_t* d_tallies,
                               const double* d_weights, double* d_T, double* d_sigmaT,
                               double* h_I_sigma, hipStream_t stream) {
    if (!valid_kernel(k) || !k->alias || !d_fine_energies || nF < 1 || !d_tallies ||
        !d_weights || !d_T || !d_sigmaT || !h_I_sigma || inject_lead > 1)
        return MCNEGF_EINVAL;
    hipError_t err = launch_interp_current(*k, d_fine_energies, (uint32_t)nF, inject_lead,
                                           d_tallies, d_weights, d_T, d_sigmaT, stream);
    if (err != hipSuccess) return hip_fail(err);
    double host[2];
    uint32_t flags = 0;
    if ((err = hipMemcpyAsync(host, k->reduce, sizeof(host), hipMemcpyDeviceToHost, stream)) !=
        hipSuccess)
        return hip_fail(err);
    if ((err = hipMemcpyAsync(&flags, k->status, sizeof(flags), hipMemcpyDeviceToHost, stream)) !=
        hipSuccess)
        return hip_fail(err);
    if ((err = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(err);
    h_I_sigma[0] = host[0];
    h_I_sigma[1] = std::sqrt(host[1] > 0.0 ? host[1] : 0.0);
    if (flags & MCNEGF_FLAG_RANGE) return MCNEGF_EINVAL;
    return status_to_code(flags, true);
}

// ---- importance-sampled walks (Sec. V A, "Improved estimator") ------------------------

struct WeightedTables {
    uint64_t off_lo, off_rho, bytes;
};

static WeightedTables weighted_tables_layout(const mcnegf_kernel& k) {
    WeightedTables t;
    const uint64_t entries = (uint64_t)k.nE * (uint64_t)k.n_out * (uint64_t)k.alias_pitch;
    t.off_lo = align256(entries * 4);
    t.off_rho = t.off_lo + align256(entries * 2);
    t.bytes = t.off_rho + align256((uint64_t)k.nE * (uint64_t)k.n_out * 8);
    return t;
}

// The modified tables need the kernel rows' ingredients (|G|^2, the exit weights, the lead
// terms), not the kernel's own tables: a kernel built with MCNEGF_BUILD_NO_ALIAS will do.
static bool valid_weighted_kernel(const mcnegf_kernel* k) {
    return valid_kernel(k) && k->wL && k->wR && k->gamma && k->Adiag && k->gam_lead &&
           k->alias_pitch >= k->n_out && k->alias_pitch % 16 == 0;
}

int32_t mc_negf_weighted_tables_bytes(const mcnegf_kernel* k, uint64_t* bytes_out) {
    if (!valid_weighted_kernel(k) || !bytes_out) return MCNEGF_EINVAL;
    *bytes_out = weighted_tables_layout(*k).bytes;
    return MCNEGF_OK;
}

int32_t mc_negf_weighted_tables(const mcnegf_kernel* k, const double* d_bias, void* d_tables,
                                uint64_t tables_bytes, hipStream_t stream) {
    if (!valid_weighted_kernel(k) || !d_bias || !d_tables) return MCNEGF_EINVAL;
    const WeightedTables t = weighted_tables_layout(*k);
    if (((uintptr_t)d_tables & 255u) != 0 || tables_bytes < t.bytes) return MCNEGF_EWS;
    char* base = static_cast<char*>(d_tables);
    hipError_t err = launch_alias_bias(*k, d_bias, reinterpret_cast<uint32_t*>(base),
                                       reinterpret_cast<uint16_t*>(base + t.off_lo),
                                       reinterpret_cast<double*>(base + t.off_rho), stream);
    return err == hipSuccess ? MCNEGF_OK : hip_fail(err);
}

int32_t mc_negf_walk_weighted_bytes(const mcnegf_kernel* k, uint64_t n_walkers,
                                    uint64_t* bytes_out) {
    if (!valid_weighted_kernel(k) || !bytes_out || n_walkers >= 0x100000000ull)
        return MCNEGF_EINVAL;
    *bytes_out = weighted_scratch_bytes(k->nE, n_walkers);
    return MCNEGF_OK;
}

int32_t mc_negf_walk_weighted(const mcnegf_kernel* k, const void* d_tables, uint64_t tables_bytes,
                              const double* d_bias, uint64_t seed, uint32_t realization,
                              uint32_t inject_lead, uint64_t walker_begin, uint64_t n_walkers,
                              uint32_t max_steps, int64_t* d_tallies, double* d_wsum,
                              void* d_scratch, uint64_t scratch_bytes, hipStream_t stream) {
    if (!valid_weighted_kernel(k) || !d_tables || !d_bias || !d_tallies || !d_wsum ||
        !d_scratch || inject_lead > 1 || realization >= (1u << 30) || max_steps < 1)
        return MCNEGF_EINVAL;
    if (walker_begin >= 0x100000000ull || n_walkers >= 0x100000000ull ||
        walker_begin + n_walkers >= 0x100000000ull)
        return MCNEGF_EINVAL;
    const WeightedTables t = weighted_tables_layout(*k);
    if (((uintptr_t)d_tables & 255u) != 0 || tables_bytes < t.bytes) return MCNEGF_EWS;
    if (((uintptr_t)d_scratch & 255u) != 0 ||
        scratch_bytes < weighted_scratch_bytes(k->nE, n_walkers))
        return MCNEGF_EWS;
    if (n_walkers == 0) return MCNEGF_OK;
    const char* base = static_cast<const char*>(d_tables);
    const uint32_t tag = (realization << 1) | inject_lead;
    hipError_t err = launch_walk_weighted(
        *k, reinterpret_cast<const uint32_t*>(base),
        reinterpret_cast<const uint16_t*>(base + t.off_lo),
        reinterpret_cast<const double*>(base + t.off_rho), d_bias, seed, tag,
        (uint32_t)walker_begin, (uint32_t)n_walkers, max_steps, d_tallies, d_wsum,
        static_cast<double*>(d_scratch), stream);
    return err == hipSuccess ? MCNEGF_OK : hip_fail(err);
}

int32_t mc_negf_current_weighted(const mcnegf_kernel* k, uint32_t inject_lead,
                                 const int64_t* d_tallies, const double* d_wsum,
                                 const double* d_weights, double* d_T, double* d_sigmaT,
                                 double* h_I_sigma, hipStream_t stream) {
    if (!valid_kernel(k) || !d_tallies || !d_wsum || !d_weights || !d_T || !d_sigmaT ||
        !h_I_sigma || inject_lead > 1)
        return MCNEGF_EINVAL;
    hipError_t err = launch_weighted_current(*k, inject_lead, d_tallies, d_wsum, d_weights, d_T,
                                             d_sigmaT, stream);
    if (err != hipSuccess) return hip_fail(err);
    double host[2];
    uint32_t flags = 0;
    if ((err = hipMemcpyAsync(host, k->reduce, sizeof(host), hipMemcpyDeviceToHost, stream)) !=
        hipSuccess)
        return hip_fail(err);
    if ((err = hipMemcpyAsync(&flags, k->status, sizeof(flags), hipMemcpyDeviceToHost, stream)) !=
        hipSuccess)
        return hip_fail(err);
    if ((err = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(err);
    h_I_sigma[0] = host[0];
    h_I_sigma[1] = std::sqrt(host[1] > 0.0 ? host[1] : 0.0);
    return status_to_code(flags, true);
}

static bool batch_units(const mcnegf_kernel* kernels, int32_t n, uint64_t* units) {
    if (!kernels || n < 1) return false;
    uint64_t u = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (!valid_kernel(&kernels[i]) || !kernels[i].alias || !kernels[i].alias_lo) return false;
        u += (uint64_t)kernels[i].nE;
    }
    if (u >= (1ull << 31)) return false;
    *units = u;
    return true;
}

static uint64_t batch_table_bytes(uint64_t units) { return align256(units * walk_unit_bytes()); }

int32_t mc_negf_batch_bytes(const mcnegf_kernel* kernels, int32_t n_kernels, uint64_t* bytes_out) {
    uint64_t units = 0;
    if (!bytes_out || !batch_units(kernels, n_kernels, &units)) return MCNEGF_EINVAL;
    *bytes_out = batch_table_bytes(units) + align256(units * MCNEGF_TALLY_N * 8);
    return MCNEGF_OK;
}

int32_t mc_negf_batch_prepare(const mcnegf_kernel* kernels, int32_t n_kernels,
                              const uint32_t* realizations, uint32_t inject_lead,
                              int64_t* const* d_tallies, void* d_buf, uint64_t buf_bytes,
                              mcnegf_batch* out, hipStream_t stream) {
    uint64_t units = 0;
    if (!batch_units(kernels, n_kernels, &units) || !realizations || !d_tallies || !d_buf ||
        !out || inject_lead > 1)
        return MCNEGF_EINVAL;
    for (int32_t i = 0; i < n_kernels; ++i)
        if (!d_tallies[i] || realizations[i] >= (1u << 30)) return MCNEGF_EINVAL;
    if (((uintptr_t)d_buf & 255u) != 0) return MCNEGF_EWS;
    const uint64_t table = batch_table_bytes(units);
    if (buf_bytes < table + align256(units * MCNEGF_TALLY_N * 8)) return MCNEGF_EWS;
    const size_t ub = walk_unit_bytes();
    std::vector<unsigned char> host(units * ub);
    uint64_t u = 0;
    for (int32_t i = 0; i < n_kernels; ++i) {
        const uint32_t tag = (realizations[i] << 1) | inject_lead;
        for (int32_t e = 0; e < kernels[i].nE; ++e, ++u)
            fill_walk_unit(host.data() + u * ub, kernels[i], e, tag, d_tallies[i]);
    }
    hipError_t err;
    if ((err = hipMemcpyAsync(d_buf, host.data(), host.size(), hipMemcpyHostToDevice, stream)) !=
        hipSuccess)
        return hip_fail(err);
    if ((err = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(err);
    out->d_units = d_buf;
    out->d_scratch_tallies = reinterpret_cast<int64_t*>(static_cast<char*>(d_buf) + table);
    out->n_units = (uint32_t)units;
    out->n_kernels = (uint32_t)n_kernels;
    return MCNEGF_OK;
}

static bool valid_walk_config(const mcnegf_walk_config& c) {
    if (c.slots < 1 || c.slots > 4) return false;
    if (c.wg_size != 64 && c.wg_size != 128 && c.wg_size != 256 && c.wg_size != 512) return false;
    if (c.groups != 1 && c.groups != 8) return false;
    if (c.chunk < 0 || (c.chunk == 0 && (c.walks_per_slot < 1 || c.walks_per_slot > 4096)))
        return false;
    return true;
}

static mcnegf_walk_config default_walk_config() {
    mcnegf_walk_config c;
    c.slots = 3;
    c.wg_size = 256;
    c.groups = 8;
    c.walks_per_slot = 8;
    c.chunk = 0;
    return c;
}

static bool valid_batch(const mcnegf_batch* b) {
    return b && b->d_units && b->d_scratch_tallies && b->n_units >= 1;
}

int32_t mc_negf_walk_batch(const mcnegf_batch* b, uint64_t seed, uint64_t walker_begin,
                           uint64_t n_walkers_per_energy, uint32_t max_steps,
                           const mcnegf_walk_config* cfg, hipStream_t stream) {
    if (!valid_batch(b) || max_steps < 1) return MCNEGF_EINVAL;
    if (walker_begin >= 0x100000000ull || n_walkers_per_energy >= 0x100000000ull ||
        walker_begin + n_walkers_per_energy >= 0x100000000ull)
        return MCNEGF_EINVAL;
    const mcnegf_walk_config c = cfg ? *cfg : default_walk_config();
    if (!valid_walk_config(c)) return MCNEGF_EINVAL;
    if (n_walkers_per_energy == 0) return MCNEGF_OK;
    hipError_t err = launch_walk_batch(*b, seed, (uint32_t)walker_begin,
                                       (uint32_t)n_walkers_per_energy, max_steps, c, nullptr,
                                       stream);
    return err == hipSuccess ? MCNEGF_OK : hip_fail(err);
}

int32_t mc_negf_walk_batch_autotune(const mcnegf_batch* b, uint64_t seed,
                                    uint64_t n_walkers_per_energy, uint32_t max_steps,
                                    mcnegf_walk_config* best, float* best_ms,
                                    hipStream_t stream) {
    if (!valid_batch(b) || !best || max_steps < 1 || n_walkers_per_energy < 1 ||
        n_walkers_per_energy > 0xffffffffull)
        return MCNEGF_EINVAL;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err;
    if ((err = hipEventCreate(&e0)) != hipSuccess) return hip_fail(err);
    if ((err = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(err);
    }
    const size_t tally_bytes = (size_t)b->n_units * MCNEGF_TALLY_N * 8;
    float best_t = -1.0f;
    mcnegf_walk_config best_c = default_walk_config();
    const int slots[] = {1, 2, 3, 4};
    const int wgs[] = {64, 256};
    const int wps[] = {2, 8, 32};
    const int groups[] = {1, 8};
    for (int sl : slots)
        for (int wg : wgs)
            for (int wp : wps)
                for (int gr : groups) {
                    mcnegf_walk_config c;
                    c.slots = sl;
                    c.wg_size = wg;
                    c.groups = gr;
                    c.walks_per_slot = wp;
                    c.chunk = 0;
                    float ms = 0.0f;
                    for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {  // warm, timed
                        err = hipMemsetAsync(b->d_scratch_tallies, 0, tally_bytes, stream);
                        if (err == hipSuccess) err = hipEventRecord(e0, stream);
                        if (err == hipSuccess)
                            err = launch_walk_batch(*b, seed, 0u, (uint32_t)n_walkers_per_energy,
                                                    max_steps, c, b->d_scratch_tallies, stream);
                        if (err == hipSuccess) err = hipEventRecord(e1, stream);
                        if (err == hipSuccess) err = hipEventSynchronize(e1);
                        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
                    }
                    if (err != hipSuccess) break;
                    if (best_t < 0.0f || ms < best_t) {
                        best_t = ms;
                        best_c = c;
                    }
                }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return hip_fail(err);
    *best = best_c;
    if (best_ms) *best_ms = best_t;
    return MCNEGF_OK;
}

int32_t mc_negf_plan_waves(const mcnegf_system* systems, int32_t n, int32_t nE,
                           uint64_t budget_bytes, int32_t* order, int32_t* wave_of,
                           int32_t* n_waves) {
    if (!systems || n < 1 || nE < 1 || !order || !wave_of || !n_waves) return MCNEGF_EINVAL;
    std::vector<uint64_t> bytes(n);
    std::vector<double> cost(n);
    for (int32_t i = 0; i < n; ++i) {
        if (!valid_system(&systems[i])) return MCNEGF_EINVAL;
        bytes[i] = layout_of(&systems[i], nE).total;
        if (bytes[i] > budget_bytes) return MCNEGF_EWS;
        const double N = (double)systems[i].W * systems[i].L;
        cost[i] = N * N * systems[i].W;
    }
    std::vector<int32_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    std::vector<uint64_t> used;
    for (int32_t k = 0; k < n; ++k) {
        const int32_t i = idx[k];
        order[k] = i;
        size_t w = 0;
        while (w < used.size() && used[w] + bytes[i] > budget_bytes) ++w;
        if (w == used.size()) used.push_back(0);
        used[w] += bytes[i];
        wave_of[i] = (int32_t)w;
    }
    *n_waves = (int32_t)used.size();
    return MCNEGF_OK;
}

}  // extern "C"

struct mcnegf_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" {

int32_t mc_negf_graph_begin(hipStream_t stream) {
    if (!stream) return MCNEGF_EINVAL;  // the legacy default stream cannot be captured
    hipError_t err = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    return err == hipSuccess ? MCNEGF_OK : hip_fail(err);
}

int32_t mc_negf_graph_end(hipStream_t stream, mcnegf_graph* out) {
    if (!stream || !out) return MCNEGF_EINVAL;
    hipGraph_t g = nullptr;
    hipError_t err = hipStreamEndCapture(stream, &g);
    if (err != hipSuccess) return hip_fail(err);
    hipGraphExec_t e = nullptr;
    if ((err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(err);
    }
    *out = new mcnegf_graph_s{g, e};
    return MCNEGF_OK;
}

int32_t mc_negf_graph_launch(mcnegf_graph g, hipStream_t stream) {
    if (!g || !stream) return MCNEGF_EINVAL;
    hipError_t err = hipGraphLaunch(g->exec, stream);
    return err == hipSuccess ? MCNEGF_OK : hip_fail(err);
}

int32_t mc_negf_graph_destroy(mcnegf_graph g) {
    if (!g) return MCNEGF_EINVAL;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
    return MCNEGF_OK;
}

}  // extern "C"
