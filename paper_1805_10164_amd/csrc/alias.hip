// Lead-to-lead transmissions and the walker's alias tables.
//
// Kernel rows (one per walker state, n = N + 2 outcomes each; states 0..N-1 are probes,
// N is lead L, N+1 is lead R):
//   probe row j : gamma_i |G_ji|^2 to probe i, <psi_j|Gamma_L|psi_j>, <psi_j|Gamma_R|psi_j>
//                 (step 6', Sec. II F, Eqs. (75), (76)); total A_jj (Sec. II D, Eq. (54));
//   lead row p  : gamma_i <psi_i|Gamma_p|psi_i> to probe i (equal to the channel marginal
//                 of steps 3-4 because G is complex symmetric), T_Lp and T_Rp to the leads;
//                 total Tr Gamma_p A (Eq. (39)).
// T_ab = Tr Gamma_a G_{ab-block} Gamma_b G^+ from the corner and diagonal blocks.
//
// Alias table of one row (Walker's method; construction by prefix sums so that a whole
// workgroup builds one row): scale the weights to mean one, s_i = w_i n / sum w.  Light
// items (s < 1) have deficit d_i = 1 - s_i, heavy items (s >= 1) surplus u_i = s_i - 1.
// Lay the deficits of the light items end to end in a fixed order (light i starts at D_i;
// thread t of the row's workgroup owns items t, t + BT, ..., and the order is by thread,
// then by item) and the surpluses of the heavy items likewise (heavy m ends at C_m); any
// fixed order gives an exact table.  Filling the light
// buckets from the heavy items in order, heavy m serves exactly the lights whose start D
// lies in [C_{m-1}, C_m); it is left with 1 + C_m - D* where D* is the first light start at
// or after C_m (or the total deficit), which becomes its own threshold, and the next heavy
// fills the rest of its bucket.  So
//   light i : threshold s_i,            alias = heavy m with C_{m-1} <= D_i < C_m,
//   heavy m : threshold 1 + C_m - D*,   alias = heavy m+1   (last heavy: threshold 1, itself).
// Each bucket c keeps outcome c with probability thr_c = floor(q_c 2^32) / 2^32 (a kept mass
// of 1 is stored as 2^32 - 1 with the bucket aliased to itself).  Storage: one 32-bit word
// per bucket with the high 16 bits of thr_c and the 16-bit alias, plus the low 16 bits of
// thr_c in a separate 16-bit array that the walker reads only on a tie of the high bits
// (probability 2^-16), so the comparison is the full 32-bit one at 4 bytes per bucket.
#include "common.h"

namespace mcnegf {

// ---------------------------------------------------------------- lead terms
__device__ inline double block_sum256(double v, double* red) {
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

// Tr Ga X Gb X^+ summed by thread (q, p): sum_{c,d} Ga[p][q] X[q][c] Gb[c][d] conj(X[p][d]).
__device__ inline double trace_term(const double2* X, const double* Ga, const double* Gb, int W,
                                    int q, int p) {
    double2 y = cmk(0.0, 0.0);
    for (int c = 0; c < W; ++c) {
        double2 xg = cmk(0.0, 0.0);
        for (int d = 0; d < W; ++d) xg = cadd(xg, cscale(cconj(X[p * W + d]), Gb[c * W + d]));
        cfma(y, X[q * W + c], xg);
    }
    return Ga[p * W + q] * y.x;
}

__global__ void __launch_bounds__(256) lead_terms_kernel(const double2* __restrict__ Gd,
                                                         const double2* __restrict__ corner,
                                                         const double* __restrict__ gam_lead,
                                                         int W, int L, double* __restrict__ lead) {
    __shared__ double red[256];
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    const double* gm = gam_lead + (size_t)e * W * W;
    const double2* G00 = Gd + (size_t)e * L * W * W;
    const double2* Gll = G00 + (size_t)(L - 1) * W * W;
    const double2* cRL = corner + (size_t)e * 2 * W * W;
    const double2* cLR = cRL + W * W;
    double tLL = 0, tRL = 0, tLR = 0, tRR = 0, aL = 0, aR = 0;
    for (int i = tid; i < W * W; i += 256) {  // thread sums of the (q, p) terms
        const int q = i / W, p = i % W;
        tLL += trace_term(G00, gm, gm, W, q, p);
        tRL += trace_term(cRL, gm, gm, W, q, p);
        tLR += trace_term(cLR, gm, gm, W, q, p);
        tRR += trace_term(Gll, gm, gm, W, q, p);
        // Tr Gamma A over the end block: A[q][p] = i (G[q][p] - conj(G[p][q]))
        const double aqp0 = -(G00[q * W + p].y + G00[p * W + q].y);
        const double aqpl = -(Gll[q * W + p].y + Gll[p * W + q].y);
        aL += gm[p * W + q] * aqp0;
        aR += gm[p * W + q] * aqpl;
    }
    const double s0 = block_sum256(tLL, red), s1 = block_sum256(tRL, red);
    const double s2 = block_sum256(tLR, red), s3 = block_sum256(tRR, red);
    const double s6 = block_sum256(aL, red), s7 = block_sum256(aR, red);
    if (tid == 0) {
        double* o = lead + (size_t)e * MCNEGF_LEAD_NTERMS;
        o[MCNEGF_LEAD_TLL] = s0;
        o[MCNEGF_LEAD_TRL] = s1;
        o[MCNEGF_LEAD_TLR] = s2;
        o[MCNEGF_LEAD_TRR] = s3;
        o[MCNEGF_LEAD_TRGLA] = s6;
        o[MCNEGF_LEAD_TRGRA] = s7;
    }
}

hipError_t launch_lead_terms(const mcnegf_kernel& k, hipStream_t s) {
    {
        MCNEGF_TIMED("lead_terms_kernel", s);
        hipLaunchKernelGGL(lead_terms_kernel, dim3(k.nE), dim3(256), 0, s,
                           reinterpret_cast<const double2*>(k.Gd),
                           reinterpret_cast<const double2*>(k.corner), k.gam_lead, k.W, k.L, k.lead);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- block reductions (BT threads)
// Sums and exclusive scans in a fixed order (lanes within a wavefront by DPP, then the
// wavefronts in order through LDS): two barriers each instead of one per tree level.
//
// Inclusive wavefront scan by data-parallel primitives: row_shr:1, 2, 4, 8 scan each row of
// 16 lanes; row_bcast:15 adds the last lane of rows 0 and 2 to rows 1 and 3; row_bcast:31
// adds lane 31 to rows 2 and 3.  A lane without a source (first lanes of a row, rows outside
// the row mask) reads the 0 given as `old`.  Every lane of the wavefront must be active.
template <int CTRL, int ROW_MASK>
__device__ inline int dpp_or_zero(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, false);
}
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_or_zero_d(double v) {
    const int lo = dpp_or_zero<CTRL, ROW_MASK>(__double2loint(v));
    const int hi = dpp_or_zero<CTRL, ROW_MASK>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

__device__ inline double wave_incl_scan(double v) {
    v += dpp_or_zero_d<kDppRowShr1, 0xF>(v);
    v += dpp_or_zero_d<kDppRowShr2, 0xF>(v);
    v += dpp_or_zero_d<kDppRowShr4, 0xF>(v);
    v += dpp_or_zero_d<kDppRowShr8, 0xF>(v);
    v += dpp_or_zero_d<kDppRowBcast15, 0xA>(v);
    v += dpp_or_zero_d<kDppRowBcast31, 0xC>(v);
    return v;
}
__device__ inline int wave_incl_scan_int(int v) {
    v += dpp_or_zero<kDppRowShr1, 0xF>(v);
    v += dpp_or_zero<kDppRowShr2, 0xF>(v);
    v += dpp_or_zero<kDppRowShr4, 0xF>(v);
    v += dpp_or_zero<kDppRowShr8, 0xF>(v);
    v += dpp_or_zero<kDppRowBcast15, 0xA>(v);
    v += dpp_or_zero<kDppRowBcast31, 0xC>(v);
    return v;
}

template <int BT>
__device__ inline double block_sum(double v, double* red) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double incl = wave_incl_scan(v);
    if (lane == 63) red[wv] = incl;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < BT / 64; ++w) r += red[w];
    __syncthreads();
    return r;
}

// Exclusive scan of one double and one int per thread, in thread order; returns totals.
template <int BT>
__device__ inline void block_scan2(double& xd, int& xi, double& totd, int& toti, double* sd,
                                   int* si) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double id = wave_incl_scan(xd);
    const int ii = wave_incl_scan_int(xi);
    if (lane == 63) {
        sd[wv] = id;
        si[wv] = ii;
    }
    __syncthreads();
    double pd = 0.0, td = 0.0;
    int pi = 0, ti = 0;
#pragma unroll
    for (int w = 0; w < BT / 64; ++w) {
        pd += w < wv ? sd[w] : 0.0;
        pi += w < wv ? si[w] : 0;
        td += sd[w];
        ti += si[w];
    }
    totd = td;
    toti = ti;
    xd = pd + id - xd;  // exclusive
    xi = pi + ii - xi;
    __syncthreads();
}

// ---------------------------------------------------------------- alias build
struct AliasArgs {
    const double* P;
    const double* wL;
    const double* wR;
    const double* Adiag;
    const double* gamma;
    double* lead;
    uint32_t* alias;     // packed (thr >> 16) << 16 | alias
    uint16_t* alias_lo;  // thr & 0xFFFF
    uint32_t* status;
    const double* gam_lead;
    int64_t ldP, pitch;
    int N, W;
    double open_cut;  // an injection row needs Tr Gamma_p > open_cut
    double rowsum_tol;  // relative tolerance of the row-total check
    // Modified rows (importance-sampled walks): outcome i of every row of energy e weighs
    // bias[e * n + i] times its kernel weight, and rho[e * n + row] receives the ratio of the
    // modified row's total to the unmodified one (0 for a row of total 0).
    const double* bias;
    double* rho;
};

// Weight of outcome i in kernel row `row` at energy e (probe rows: gamma_i |G_row,i|^2 and the
// exit weights; injection rows N, N + 1: gamma_i <psi_i|Gamma_p|psi_i> and the lead terms);
// rounding negatives are clamped to zero, a NaN is kept.
__device__ inline double kernel_weight(const AliasArgs& a, int e, int row, int i) {
    const int N = a.N;
    const double* lead = a.lead + (size_t)e * MCNEGF_LEAD_NTERMS;
    const double* wLe = a.wL + (size_t)e * N;
    const double* wRe = a.wR + (size_t)e * N;
    double v;
    if (row < N) {
        if (i < N) v = a.gamma[i] * a.P[((size_t)e * N + row) * a.ldP + i];
        else v = (i == N) ? wLe[row] : wRe[row];
    } else if (row == N) {
        if (i < N) v = a.gamma[i] * wLe[i];
        else v = (i == N) ? lead[MCNEGF_LEAD_TLL] : lead[MCNEGF_LEAD_TRL];
    } else {
        if (i < N) v = a.gamma[i] * wRe[i];
        else v = (i == N) ? lead[MCNEGF_LEAD_TLR] : lead[MCNEGF_LEAD_TRR];
    }
    return v > 0.0 ? v : (v == v ? 0.0 : v);
}

// One workgroup of BT threads per row; thread t owns the items t + BT k (k < KM, n <= BT KM)
// and keeps their weights in registers (loads coalesced across the wavefront).  LDS holds what other
// threads search: the light starts and heavy ends in one array of n + 1 doubles (lights from
// the front with the total deficit after the last one, heavies from the back: heavy m at
// n - m) and the heavy items' indices (16 bits): 10 n bytes per row.
// With kBias the row is the modified one of an importance-sampled walk (outcome i weighs
// b_i K_row,i), written to the caller's tables; rho = modified total / unmodified total is
// stored per row, the injection rows' unmodified totals c_p as the plain build stores them,
// and the row-total checks of the build are left alone.
template <int BT, int KM, bool kBias = false>
__global__ void __launch_bounds__(BT) alias_build_kernel(AliasArgs a) {
    constexpr bool kLong = KM > 8;  // rows above BT * 8 outcomes
    extern __shared__ double smem[];
    __shared__ double sd[BT / 64];  // one partial per wavefront
    __shared__ int si[BT / 64];
    const int N = a.N;
    const int n = N + 2;
    const int row = blockIdx.x;
    const int e = blockIdx.y;
    const int tid = threadIdx.x;
    double* lh = smem;                                   // [n+1] light starts | heavy ends
    // 16-bit item indices [n]: heavy m at m (rows up to BT * 8 outcomes); for longer rows
    // light r at r and heavy m at n - 1 - m
    uint16_t* idx = reinterpret_cast<uint16_t*>(lh + n + 1);
    auto lightD = [&](int r) -> double& { return lh[r]; };
    auto heavyC = [&](int m) -> double& { return lh[n - m]; };
    auto heavyIdx = [&](int m) -> uint16_t& { return kLong ? idx[n - 1 - m] : idx[m]; };

    const double* lead = a.lead + (size_t)e * MCNEGF_LEAD_NTERMS;
    // 1. weights of this row (items beyond n weigh 0 and are skipped below)
    double w[KM];
    double part0 = 0.0;  // (kBias) the unmodified row's part, in the order of part below
    bool bad_bias = false;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const int i = tid + BT * k;
        double v = i < n ? kernel_weight(a, e, row, i) : 0.0;
        if constexpr (kBias) {
            const double b = i < n ? a.bias[(size_t)e * n + i] : 0.0;
            bad_bias |= !(b >= 0.0 && b <= 1.7976931348623157e308);
            part0 += v;
            v *= b;
        }
        w[k] = v;
    }
    // 2. total (fixed order: by thread, then by item)
    double part = 0.0;
#pragma unroll
    for (int k = 0; k < KM; ++k) part += w[k];
    double total = block_sum<BT>(part, sd);
    double total0 = kBias ? block_sum<BT>(part0, sd) : total;
    if (row >= N) {
        // no open channel in this lead (outside its band, Gamma only from the regulator)
        double trg = 0.0;
        for (int y = 0; y < a.W; ++y) trg += a.gam_lead[((size_t)e * a.W + y) * a.W + y];
        if (!(trg > a.open_cut)) total = total0 = 0.0;
    }

    uint32_t* out = a.alias + ((size_t)e * n + row) * a.pitch;
    uint16_t* out_lo = a.alias_lo + ((size_t)e * n + row) * a.pitch;
    if constexpr (kBias) {
        if (tid == 0) {
            a.rho[(size_t)e * n + row] = total0 > 0.0 ? total / total0 : 0.0;
            // c_p, as the kernel's own build writes it (a kernel built without its own
            // tables has it only from here)
            if (row == N) a.lead[(size_t)e * MCNEGF_LEAD_NTERMS + MCNEGF_LEAD_CL] = total0;
            if (row == N + 1) a.lead[(size_t)e * MCNEGF_LEAD_NTERMS + MCNEGF_LEAD_CR] = total0;
            if (!isfinite(total)) atomicOr(a.status, MCNEGF_FLAG_NONFINITE);
        }
        if (bad_bias) atomicOr(a.status, MCNEGF_FLAG_NONFINITE);
    } else if (tid == 0) {
        double ref;
        if (row < N) ref = a.Adiag[(size_t)e * N + row];
        else ref = lead[row == N ? MCNEGF_LEAD_TRGLA : MCNEGF_LEAD_TRGRA];
        if (row == N) a.lead[(size_t)e * MCNEGF_LEAD_NTERMS + MCNEGF_LEAD_CL] = total;
        if (row == N + 1) a.lead[(size_t)e * MCNEGF_LEAD_NTERMS + MCNEGF_LEAD_CR] = total;
        if (!isfinite(total)) atomicOr(a.status, MCNEGF_FLAG_NONFINITE);
        else if (row < N && total > 0.0 && fabs(total - ref) > a.rowsum_tol * fabs(ref))
            atomicOr(a.status, MCNEGF_FLAG_ROWSUM);
        else if (row >= N && total > 0.0 && fabs(total - ref) > a.rowsum_tol * fabs(ref))
            atomicOr(a.status, MCNEGF_FLAG_ROWSUM);
        if (row >= N && !(total > 0.0)) atomicOr(a.status, MCNEGF_FLAG_NOABSORB);
    }
    if (!(total > 0.0) || !isfinite(total)) {
        // Degenerate row: every bucket exits at lead L (its estimator weight is zero).
        for (int i = tid; i < n; i += BT) {
            out[i] = (uint32_t)N;
            out_lo[i] = 0;
        }
        return;
    }
    // 3. scale, classify, scan
    const double scale = (double)n / total;
    double dl = 0.0, uh = 0.0;
    int nl = 0, nh = 0;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const double v = w[k] * scale;
        w[k] = v;
        if ((tid + BT * k) < n) {
            if (v < 1.0) { dl += 1.0 - v; ++nl; }
            else { uh += v - 1.0; ++nh; }
        }
    }
    double Dtot, Utot;
    int NLtot, NHtot;
    block_scan2<BT>(dl, nl, Dtot, NLtot, sd, si);
    block_scan2<BT>(uh, nh, Utot, NHtot, sd, si);
    int rk[KM];     // light rank, or ~heavy rank
    double dc[KM];  // light start D, or heavy end C
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        const int i = tid + BT * k;
        const double v = w[k];
        rk[k] = 0;
        dc[k] = 0.0;
        if (i < n) {
            if (v < 1.0) {
                lightD(nl) = dl;
                if (kLong) idx[nl] = (uint16_t)i;
                rk[k] = nl;
                dc[k] = dl;
                dl += 1.0 - v;
                ++nl;
            } else {
                uh += v - 1.0;
                heavyC(nh) = uh;
                heavyIdx(nh) = (uint16_t)i;
                rk[k] = ~nh;
                dc[k] = uh;
                ++nh;
            }
        }
    }
    if (tid == 0) lightD(NLtot) = Dtot;  // index NLtot = n - NHtot: below every heavy slot
    __syncthreads();
    // 4. thresholds and aliases.  Light r is served by heavy m*(r), the first heavy with
    // C_m > D_r (the last heavy when there is none); heavy m keeps 1 + C_m - D_a with a the
    // first light with D_a >= C_m (D_NL = the total deficit) and aliases to heavy m + 1.
    if constexpr (KM <= 8) {
        // Both are ranks in the merge of the ascending D and C with a heavy before a light on
        // ties: thread t merges positions [t KM, t KM + KM) from the split its binary search
        // finds, keeps the results of the merged items in registers and, once every merge has
        // read D and C, passes them through the lh array (one 64-bit slot per item: light r at
        // slot r, heavy m at slot n - 1 - m) to the threads that own the items.
        uint64_t res[KM];
        int slot[KM];
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            res[k] = 0;
            slot[k] = -1;
        }
        if (NHtot > 0) {
            const int d0 = tid * KM;
            int a = 0, b = 0;
            if (d0 < n) {
                int lo = d0 > NHtot ? d0 - NHtot : 0, hi = d0 < NLtot ? d0 : NLtot;
                while (lo < hi) {  // lights among the first d0 merged items
                    const int mid = (lo + hi) >> 1;
                    if (lightD(mid) < heavyC(d0 - mid - 1)) lo = mid + 1; else hi = mid;
                }
                a = lo;
                b = d0 - lo;
            }
            double dA = lightD(a);  // lightD(NLtot) = Dtot
            double cB = b < NHtot ? heavyC(b) : 0.0;
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                if (d0 + k >= n) continue;
                const bool heavy = b < NHtot && (a >= NLtot || cB <= dA);
                if (heavy) {
                    const int i = heavyIdx(b);
                    double q;
                    int al;
                    if (b == NHtot - 1) {
                        q = 1.0;
                        al = i;
                    } else {
                        q = 1.0 + cB - dA;
                        q = q < 0.0 ? 0.0 : q;
                        al = heavyIdx(b + 1);
                    }
                    uint32_t thr;
                    if (q >= 1.0) {
                        thr = 0xFFFFFFFFu;
                        al = i;
                    } else {
                        thr = (uint32_t)(q * 4294967296.0);
                    }
                    res[k] = (uint64_t)((thr & ~kAliasIdxMask) | (uint32_t)al) |
                             ((uint64_t)(thr & kAliasIdxMask) << 32);
                    slot[k] = n - 1 - b;
                    ++b;
                    cB = b < NHtot ? heavyC(b) : 0.0;
                } else {
                    res[k] = heavyIdx(b < NHtot ? b : NHtot - 1);
                    slot[k] = a;
                    ++a;
                    dA = lightD(a);
                }
            }
        }
        __syncthreads();  // every merge has read D and C
        uint64_t* slots = reinterpret_cast<uint64_t*>(lh);
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (slot[k] >= 0) slots[slot[k]] = res[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const int i = tid + BT * k;
            if (i >= n) continue;
            const int r = rk[k];
            uint32_t packed, low;
            if (NHtot == 0) {
                packed = (0xFFFFFFFFu & ~kAliasIdxMask) | (uint32_t)i;
                low = 0xFFFFFFFFu & kAliasIdxMask;
            } else if (r >= 0) {
                int al = (int)slots[r];
                uint32_t thr;
                if (w[k] >= 1.0) {
                    thr = 0xFFFFFFFFu;
                    al = i;
                } else {
                    thr = (uint32_t)(w[k] * 4294967296.0);
                }
                packed = (thr & ~kAliasIdxMask) | (uint32_t)al;
                low = thr & kAliasIdxMask;
            } else {
                const uint64_t v = slots[n - 1 - ~r];
                packed = (uint32_t)v;
                low = (uint32_t)(v >> 32);
            }
            if ((packed & kAliasIdxMask) >= (uint32_t)n) {  // never for a consistent row
                packed = (packed & ~kAliasIdxMask) | (uint32_t)i;
                atomicOr(a.status, MCNEGF_FLAG_NONFINITE);
            }
            out[i] = packed;
            out_lo[i] = (uint16_t)low;
        }
    } else {
        // Long rows: the same merge with the 16-bit item indices of lights and heavies in LDS
        // (a light keeps 1 - (D_{r+1} - D_r), its own deficit recovered from the starts).  The
        // merged results wait in registers (the row's weights, ranks and prefix values are no
        // longer needed) until every merge has read D and C, then go through the lh array by
        // item index (one 64-bit slot per item) to the threads that own the items, which write
        // coalesced entries.
        if (NHtot == 0) {
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const int i = tid + BT * k;
                if (i < n) {
                    out[i] = (0xFFFFFFFFu & ~kAliasIdxMask) | (uint32_t)i;
                    out_lo[i] = (uint16_t)(0xFFFFFFFFu & kAliasIdxMask);
                }
            }
            return;  // uniform: NHtot is the block's total
        }
        uint64_t res[KM];
        int itm[KM];  // item of each merged result (-1: none)
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            res[k] = 0;
            itm[k] = -1;
        }
        const int d0 = tid * KM;
        if (d0 < n) {
            int lo = d0 > NHtot ? d0 - NHtot : 0, hi = d0 < NLtot ? d0 : NLtot;
            while (lo < hi) {  // lights among the first d0 merged items
                const int mid = (lo + hi) >> 1;
                if (lightD(mid) < heavyC(d0 - mid - 1)) lo = mid + 1; else hi = mid;
            }
            int ra = lo, rb = d0 - lo;
            double dA = lightD(ra);  // lightD(NLtot) = Dtot
            double cB = rb < NHtot ? heavyC(rb) : 0.0;
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                if (d0 + k >= n) continue;
                const bool heavy = rb < NHtot && (ra >= NLtot || cB <= dA);
                int i, al;
                double q;
                if (heavy) {
                    i = heavyIdx(rb);
                    if (rb == NHtot - 1) {
                        q = 1.0;
                        al = i;
                    } else {
                        q = 1.0 + cB - dA;
                        q = q < 0.0 ? 0.0 : q;
                        al = heavyIdx(rb + 1);
                    }
                    ++rb;
                    cB = rb < NHtot ? heavyC(rb) : 0.0;
                } else {
                    i = idx[ra];
                    const double dn = lightD(ra + 1);
                    q = 1.0 - (dn - dA);
                    q = q < 0.0 ? 0.0 : q;
                    al = heavyIdx(rb < NHtot ? rb : NHtot - 1);
                    ++ra;
                    dA = dn;
                }
                uint32_t thr;
                if (q >= 1.0) {
                    thr = 0xFFFFFFFFu;
                    al = i;
                } else {
                    thr = (uint32_t)(q * 4294967296.0);
                }
                if ((unsigned)al >= (unsigned)n || (unsigned)i >= (unsigned)n) {
                    // never for a consistent row; keeps walks and stores in range
                    atomicOr(a.status, MCNEGF_FLAG_NONFINITE);
                    if ((unsigned)i >= (unsigned)n) continue;
                    al = i;
                }
                res[k] = (uint64_t)((thr & ~kAliasIdxMask) | (uint32_t)al) |
                         ((uint64_t)(thr & kAliasIdxMask) << 32);
                itm[k] = i;
            }
        }
        __syncthreads();  // every merge has read D and C
        uint64_t* slots = reinterpret_cast<uint64_t*>(lh);
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (itm[k] >= 0) slots[itm[k]] = res[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const int i = tid + BT * k;
            if (i < n) {
                const uint64_t v = slots[i];
                out[i] = (uint32_t)v;
                out_lo[i] = (uint16_t)(v >> 32);
            }
        }
    }
}

// ---------------------------------------------------------------- interpolation check
// For each pair of neighbouring energies (e, e + 1) of a build: the largest, over the kernel
// rows, L1 distance between the two normalised rows, sum_i |w_i(e) / W(e) - w_i(e+1) / W(e+1)|
// (Sec. V A, "Interpolation": where the probabilities at two nearby energies differ little,
// those between them are interpolated linearly).  One workgroup per (row, pair); rows are
// combined by an integer max on the bit pattern (non-negative doubles order as their bits).
// A row with a total that is not positive and finite counts as distance 2 (the largest).
__global__ void __launch_bounds__(256) interp_distance_kernel(AliasArgs a,
                                                              unsigned long long* dist) {
    __shared__ double sd[4];
    const int n = a.N + 2;
    const int row = blockIdx.x;
    const int e = blockIdx.y;
    double t0 = 0.0, t1 = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        t0 += kernel_weight(a, e, row, i);
        t1 += kernel_weight(a, e + 1, row, i);
    }
    t0 = block_sum<256>(t0, sd);
    t1 = block_sum<256>(t1, sd);
    double d = 2.0;
    if (t0 > 0.0 && t1 > 0.0 && isfinite(t0) && isfinite(t1)) {
        const double r0 = 1.0 / t0, r1 = 1.0 / t1;
        double part = 0.0;
        for (int i = threadIdx.x; i < n; i += 256)
            part += fabs(kernel_weight(a, e, row, i) * r0 - kernel_weight(a, e + 1, row, i) * r1);
        d = block_sum<256>(part, sd);
    }
    if (threadIdx.x == 0) atomicMax(dist + e, (unsigned long long)__double_as_longlong(d));
}

__global__ void fill_u64_kernel(unsigned long long* p, int n, unsigned long long v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static AliasArgs alias_args(const mcnegf_kernel& k, double rowsum_tol) {
    AliasArgs a;
    a.P = k.P;
    a.wL = k.wL;
    a.wR = k.wR;
    a.Adiag = k.Adiag;
    a.gamma = k.gamma;
    a.lead = k.lead;
    a.alias = k.alias;
    a.alias_lo = k.alias_lo;
    a.status = k.status;
    a.gam_lead = k.gam_lead;
    a.ldP = k.p_pitch;
    a.pitch = k.alias_pitch;
    a.N = k.N;
    a.W = k.W;
    a.open_cut = 1e3 * k.delta_lead * k.t * k.W;
    a.rowsum_tol = rowsum_tol;
    a.bias = nullptr;
    a.rho = nullptr;
    return a;
}

hipError_t launch_interp_distances(const mcnegf_kernel& k, double* dist, hipStream_t s) {
    const int pairs = k.nE - 1;
    if (pairs < 1) return hipSuccess;
    unsigned long long* d = reinterpret_cast<unsigned long long*>(dist);
    {
        MCNEGF_TIMED("fill_u64_kernel", s);
        hipLaunchKernelGGL(fill_u64_kernel, dim3((pairs + 255) / 256), dim3(256), 0, s, d, pairs,
                           0ull);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    {
        MCNEGF_TIMED("interp_distance_kernel", s);
        hipLaunchKernelGGL(interp_distance_kernel, dim3(k.n_out, pairs), dim3(256), 0, s,
                           alias_args(k, 0.0), d);
    }
    return hipGetLastError();
}

// Alias tables of every row of every energy from the arguments a (the kernel's own tables,
// or with kBias the modified rows into the caller's tables).
template <bool kBias>
static hipError_t launch_alias_rows(const mcnegf_kernel& k, const AliasArgs& a,
                                    const char* name, hipStream_t s) {
    const int n = k.n_out;
    const size_t lds = (size_t)(n + 1) * 8 + (size_t)n * 2;
    // rows up to 1024 outcomes: 128 threads x 8 items; up to 1536: 256 x 6; up to 4096:
    // 512 x 8; up to 8192: 512 x 16; longer rows (n <= kMaxOut): 512 x 32
    const int shape = n <= 128 * 8 ? 0 : n <= 256 * 6 ? 1 : n <= 512 * 8 ? 2 : n <= 512 * 16 ? 3 : 4;
    const void* fns[5] = {(const void*)alias_build_kernel<128, 8, kBias>,
                          (const void*)alias_build_kernel<256, 6, kBias>,
                          (const void*)alias_build_kernel<512, 8, kBias>,
                          (const void*)alias_build_kernel<512, 16, kBias>,
                          (const void*)alias_build_kernel<512, 32, kBias>};
    const int bts[5] = {128, 256, 512, 512, 512};
    if (lds > 65536) {
        // rows beyond 6.5k outcomes need more than 64 KB of LDS per workgroup (gfx950: 160 KB)
        int dev = 0, per_block = 0, optin = 0;
        hipError_t err = hipGetDevice(&dev);
        if (err == hipSuccess)
            err = hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (err != hipSuccess) return err;
        if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) !=
            hipSuccess) {
            optin = 0;
            (void)hipGetLastError();  // the launch below reports its own error
        }
        const int max_lds = optin > per_block ? optin : per_block;
        hipFuncAttributes fa;
        if ((err = hipFuncGetAttributes(&fa, fns[shape])) != hipSuccess) return err;
        if (lds + fa.sharedSizeBytes > (size_t)max_lds) return hipErrorInvalidConfiguration;
        err = hipFuncSetAttribute(fns[shape], hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (err != hipSuccess) return err;
    }
    {
        MCNEGF_TIMED(name, s);
        const dim3 grid(n, k.nE), block(bts[shape]);
        switch (shape) {
            case 0: hipLaunchKernelGGL((alias_build_kernel<128, 8, kBias>), grid, block, lds, s, a); break;
            case 1: hipLaunchKernelGGL((alias_build_kernel<256, 6, kBias>), grid, block, lds, s, a); break;
            case 2: hipLaunchKernelGGL((alias_build_kernel<512, 8, kBias>), grid, block, lds, s, a); break;
            case 3: hipLaunchKernelGGL((alias_build_kernel<512, 16, kBias>), grid, block, lds, s, a); break;
            default: hipLaunchKernelGGL((alias_build_kernel<512, 32, kBias>), grid, block, lds, s, a); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_alias_build(const mcnegf_kernel& k, double rowsum_tol, hipStream_t s) {
    return launch_alias_rows<false>(k, alias_args(k, rowsum_tol), "alias_build_kernel", s);
}

hipError_t launch_alias_bias(const mcnegf_kernel& k, const double* bias, uint32_t* tables,
                             uint16_t* lows, double* rho, hipStream_t s) {
    AliasArgs a = alias_args(k, 0.0);
    a.alias = tables;
    a.alias_lo = lows;
    a.bias = bias;
    a.rho = rho;
    return launch_alias_rows<true>(k, a, "alias_bias_kernel", s);
}

}  // namespace mcnegf
