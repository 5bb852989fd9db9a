// All blocks of G^r from the RGF blocks, streamed straight into the walker's weights.
//
// For a column l (slice of the column), the blocks of G obey (E - H - Sigma) G = I with
// off-diagonal blocks t I, which gives
//   above the diagonal  G_{k,l} = -t gL_k G_{k+1,l}   (k < l),
//   below the diagonal  G_{k,l} = -t gR_k G_{k-1,l}   (k > l),
// starting from the diagonal block G_{l,l}.  Each lane owns one column j of G (a workgroup
// is one wavefront owning 64 consecutive columns) and keeps its W-vector G_{k, j} in
// registers while the wavefront sweeps k down and then up the wire; the W x W factors gL_k,
// gR_k are the same for every lane: the wavefront stages them in LDS one slice ahead
// (double-buffered) and every lane reads the same address (a broadcast), which keeps the
// block operands off the scalar path and the texture units.  Nothing of G is written except
//   P[i][j]  = |G_ij|^2                      (probe-to-probe weights, step 6', Eq. (75)),
//   wL[j]    = <psi_j|Gamma_L|psi_j>, wR[j]  (psi_j = G|j>, exit weights, Eq. (76)),
//   corner   = G_{L-1,0} and G_{0,L-1}       (lead-to-lead transmissions).
// Rows of P are written by 64 lanes at consecutive columns (coalesced 512-byte segments).
// The block products run on the FP64 VALU: the operands live in registers and LDS, and
// gfx950's FP64 matrix-core rate equals its FP64 FMA rate, so padding W up to a 16x16x4 MFMA
// shape would only add work.  Up to W = 24 the column and the product fit the register file;
// at W = 32 a few values spill.
#include "common.h"

namespace mcnegf {

template <int W>
__device__ inline double quad_form(const double2 (&v)[W], const double* __restrict__ gm) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < W; ++a) {
#pragma unroll
        for (int b = 0; b < W; ++b)
            acc = fma(gm[a * W + b], v[a].x * v[b].x + v[a].y * v[b].y, acc);
    }
    return acc;
}

typedef __attribute__((address_space(3))) double lds_double;

// v <- mt * M v for a W x W complex block M staged in LDS as (re, im) pairs, row-major.
template <int W>
__device__ inline void block_matvec(double2 (&v)[W], const lds_double* M, double mt) {
    double2 nv[W];
#pragma unroll
    for (int y = 0; y < W; ++y) {
        double2 acc = cmk(0.0, 0.0);
#pragma unroll
        for (int x = 0; x < W; ++x) cfma(acc, cmk(M[2 * (y * W + x)], M[2 * (y * W + x) + 1]), v[x]);
        nv[y] = cscale(acc, mt);
    }
#pragma unroll
    for (int y = 0; y < W; ++y) v[y] = nv[y];
}

// The NT threads copy the W x W block src into the LDS buffer dst (thread tid).
template <int W, int NT = 64>
__device__ inline void stage_block(lds_double* dst, const double2* __restrict__ src, int tid) {
#pragma unroll
    for (int i = tid; i < W * W; i += NT) {
        const double2 v = src[i];
        dst[2 * i] = v.x;
        dst[2 * i + 1] = v.y;
    }
}

// STORE_G: write the complex blocks of G (row-major, pitch ldG, Gc) instead of |G_ij|^2,
// the exit weights and the corners.
template <int W, bool STORE_G>
__global__ void __launch_bounds__(64) fullinv_kernel(const double2* __restrict__ gL,
                                                      const double2* __restrict__ gR,
                                                      const double2* __restrict__ Gd,
                                                      const double* __restrict__ gam_lead,
                                                      int L, double t, int64_t ldP,
                                                      double* __restrict__ P,
                                                      double* __restrict__ wL,
                                                      double* __restrict__ wR,
                                                      double2* __restrict__ corner,
                                                      double2* __restrict__ Gc, int64_t ldG,
                                                      int nE) {
    const int N = W * L;
    // XCD-aware order: workgroups are dealt to the eight XCDs in turn (workgroup b on XCD
    // b % 8); every column tile of energy e runs on XCD e % 8, whose L2 then fetches that
    // energy's RGF blocks once for all its tiles
    const int tiles = (N + 63) / 64;
    const int xcd = blockIdx.x & 7, jb = blockIdx.x >> 3;
    const int e = xcd + 8 * (jb / tiles);
    if (e >= nE) return;  // padding of the last round (whole workgroup)
    const int lane = threadIdx.x;
    const int wave_first = (jb % tiles) * 64;
    const int col = wave_first + lane;
    const bool valid = col < N;
    const int colc = valid ? col : N - 1;
    const int l = colc / W;
    const int y0 = colc - l * W;
    const int wave_last = min(wave_first + 63, N - 1);
    const int kmin = wave_first / W;
    const int kmax = wave_last / W;
    const size_t eb = (size_t)e * L * W * W;
    const double2* gLe = gL + eb;
    const double2* gRe = gR + eb;
    const double2* Gde = Gd + eb;
    const double* gme = gam_lead + (size_t)e * W * W;
    double* Pe = P + (size_t)e * N * ldP;
    double2* cRL = corner + (size_t)e * 2 * W * W;
    double2* cLR = cRL + W * W;
    const double mt = -t;
    constexpr int BS = 2 * W * W;  // doubles per staged block
    __shared__ double Ms_raw[2 * BS];
    lds_double* Ms = (lds_double*)Ms_raw;

    double2 v[W];
    // ---- downward: k = l, l+1, ..., L-1 -------------------------------------------------
#pragma unroll
    for (int y = 0; y < W; ++y) v[y] = cmk(0.0, 0.0);
    stage_block<W>(Ms, gRe + (size_t)kmin * W * W, lane);
    for (int k = kmin; k < L; ++k) {
        __syncthreads();  // block k staged; the other buffer is free
        const int b = (k - kmin) & 1;
        if (k + 1 < L) stage_block<W>(Ms + (b ^ 1) * BS, gRe + (size_t)(k + 1) * W * W, lane);
        block_matvec<W>(v, Ms + b * BS, mt);
        if (k == l) {
#pragma unroll
            for (int y = 0; y < W; ++y) v[y] = Gde[(size_t)k * W * W + y * W + y0];
        }
        if (k < l) {
#pragma unroll
            for (int y = 0; y < W; ++y) v[y] = cmk(0.0, 0.0);
        }
        if (valid && k >= l) {
            if (STORE_G) {
                double2* Ge = Gc + (size_t)e * N * ldG;
#pragma unroll
                for (int y = 0; y < W; ++y) Ge[(size_t)(k * W + y) * ldG + col] = v[y];
            } else {
#pragma unroll
                for (int y = 0; y < W; ++y) Pe[(size_t)(k * W + y) * ldP + col] = cabs2(v[y]);
            }
        }
    }
    // k = L-1 now: exit weight into R and, for columns of slice 0, the corner G_{L-1,0}.
    if (valid && !STORE_G) {
        wR[(size_t)e * N + col] = quad_form<W>(v, gme);
        if (l == 0) {
#pragma unroll
            for (int y = 0; y < W; ++y) cRL[y * W + y0] = v[y];
        }
    }
    // ---- upward: k = l, l-1, ..., 0 ------------------------------------------------------
#pragma unroll
    for (int y = 0; y < W; ++y) v[y] = cmk(0.0, 0.0);
    __syncthreads();  // downward reads done
    stage_block<W>(Ms, gLe + (size_t)kmax * W * W, lane);
    for (int k = kmax; k >= 0; --k) {
        __syncthreads();
        const int b = (kmax - k) & 1;
        if (k > 0) stage_block<W>(Ms + (b ^ 1) * BS, gLe + (size_t)(k - 1) * W * W, lane);
        block_matvec<W>(v, Ms + b * BS, mt);
        if (k == l) {
#pragma unroll
            for (int y = 0; y < W; ++y) v[y] = Gde[(size_t)k * W * W + y * W + y0];
        }
        if (k > l) {
#pragma unroll
            for (int y = 0; y < W; ++y) v[y] = cmk(0.0, 0.0);
        }
        if (valid && k < l) {
            if (STORE_G) {
                double2* Ge = Gc + (size_t)e * N * ldG;
#pragma unroll
                for (int y = 0; y < W; ++y) Ge[(size_t)(k * W + y) * ldG + col] = v[y];
            } else {
#pragma unroll
                for (int y = 0; y < W; ++y) Pe[(size_t)(k * W + y) * ldP + col] = cabs2(v[y]);
            }
        }
    }
    if (valid && !STORE_G) {
        wL[(size_t)e * N + col] = quad_form<W>(v, gme);
        if (l == L - 1) {
#pragma unroll
            for (int y = 0; y < W; ++y) cLR[y * W + y0] = v[y];
        }
    }
}

template <int W, bool STORE_G>
static hipError_t launch_fullinv_w(const mcnegf_kernel& k, double2* Gc, int64_t ldG,
                                   hipStream_t s) {
    const unsigned tiles = (unsigned)((k.N + 63) / 64);
    dim3 grid(8u * tiles * (unsigned)((k.nE + 7) / 8));
    {
        MCNEGF_TIMED(STORE_G ? "fullinv_store_g_kernel" : "fullinv_kernel", s);
        hipLaunchKernelGGL((fullinv_kernel<W, STORE_G>), grid, dim3(64), 0, s,
                           reinterpret_cast<const double2*>(k.gL),
                           reinterpret_cast<const double2*>(k.gR),
                           reinterpret_cast<const double2*>(k.Gd), k.gam_lead, k.L, k.t, k.p_pitch,
                           k.P, k.wL, k.wR, reinterpret_cast<double2*>(k.corner), Gc, ldG,
                           k.nE);
    }
    return hipGetLastError();
}

// ---- W = 16 and W = 32 on FP64 matrix cores ----------------------------------------------
//
// The same sweeps, with the block products on v_mfma_f64_16x16x4f64 (no padding at these
// widths).  A workgroup of NW wavefronts shares one double-buffered staged block (so the LDS of
// a workgroup does not limit the wavefronts a CU holds) and sweeps from its first column's
// slice (downward) and its last column's slice (upward); a wavefront's columns stay zero until
// their own slice.  A wavefront owns TC tiles of 16 consecutive columns; lane (n, g) = (l % 16, l / 16)
// holds, for tile t and row tile rt, the rows 16 rt + 4 r + g (r = 0..3) of column n, which is
// both the accumulator layout of the product (item r of lane n + 16 g is row 4 r + g) and the
// B-operand layout of the next product (K-step s takes rows 4 s + g from lane n + 16 g), so the
// columns stay in registers from slice to slice.  The A operand of K-step s and row tile rt,
// lane (m, g): (-t) M[16 rt + m][4 s + g], read from the LDS-staged block.  A complex product
// is four real products (re re, -im im into the real part; re im, im re into the imaginary).
typedef double dmfma4 __attribute__((ext_vector_type(4)));
typedef float fmfma4 __attribute__((ext_vector_type(4)));

// One 16x16x4 product on the matrix cores in the column state's precision.
__device__ inline dmfma4 mfma4(double a, double b, dmfma4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline fmfma4 mfma4(float a, float b, fmfma4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct Mfma4;
template <> struct Mfma4<double> { typedef dmfma4 type; };
template <> struct Mfma4<float> { typedef fmfma4 type; };

// Row of item r in lane group g within a 16-row tile: the FP64 product returns row 4 r + g,
// the FP32 product row 4 g + r.  In both cases K-step s of the next product takes item
// s & 3 of tile s >> 2 from every lane group, i.e. the contraction runs over the rows in the
// order the accumulator holds them, and the A operand is read in that column order.
template <typename T>
__device__ inline int tile_row(int r, int g) {
    return sizeof(T) == 8 ? 4 * r + g : 4 * g + r;
}

// T = double: FP64 products throughout.  T = float (a build with FP32 block products): the
// column state and the products are FP32 (the staged FP64 blocks are rounded as they are
// read), |G|^2, the exit weights and the corners are formed from the FP32 state in FP64.
template <int W, int TC, int NW, bool STORE_G, typename T = double>
__global__ void __launch_bounds__(64 * NW) fullinv_mfma_kernel(const double2* __restrict__ gL,
                                                          const double2* __restrict__ gR,
                                                          const double2* __restrict__ Gd,
                                                          const double* __restrict__ gam_lead,
                                                          int L, double t, int64_t ldP,
                                                          double* __restrict__ P,
                                                          double* __restrict__ wL,
                                                          double* __restrict__ wR,
                                                          double2* __restrict__ corner,
                                                          double2* __restrict__ Gc, int64_t ldG) {
    constexpr int RT = W / 16;  // row tiles
    constexpr int S = W / 4;    // K-steps
    constexpr int BS = 2 * W * W;
    __shared__ double Ms_raw[2 * BS];
    lds_double* Ms = (lds_double*)Ms_raw;
    const int N = W * L;
    const int e = blockIdx.y;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int n = lane & 15, g = lane >> 4;
    const int cg0 = blockIdx.x * NW * 16 * TC;  // the workgroup's first column
    const int c0 = cg0 + (tid >> 6) * 16 * TC;  // this wavefront's first column
    const int kmin = cg0 / W;
    const int kmax = (min(cg0 + NW * 16 * TC, N) - 1) / W;
    const size_t eb = (size_t)e * L * W * W;
    const double2* gLe = gL + eb;
    const double2* gRe = gR + eb;
    const double2* Gde = Gd + eb;
    const double* gme = gam_lead + (size_t)e * W * W;
    double* Pe = P + (size_t)e * N * ldP;
    double2* cRL = corner + (size_t)e * 2 * W * W;
    double2* cLR = cRL + W * W;
    double2* Ge = Gc + (size_t)e * N * ldG;
    const double mt = -t;

    int col[TC], l[TC], y0[TC];
    bool valid[TC];
#pragma unroll
    for (int tc = 0; tc < TC; ++tc) {
        col[tc] = c0 + 16 * tc + n;
        valid[tc] = col[tc] < N;
        const int cc = valid[tc] ? col[tc] : N - 1;
        l[tc] = cc / W;
        y0[tc] = cc - l[tc] * W;
    }
    typedef typename Mfma4<T>::type acc4;
    T vr[TC][RT][4], vi[TC][RT][4];

    // one slice: v <- (-t) M v with M the block staged at buf
    auto product = [&](const lds_double* buf) {
        acc4 cr[TC][RT], ci[TC][RT];
#pragma unroll
        for (int tc = 0; tc < TC; ++tc)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                cr[tc][rt] = acc4{0, 0, 0, 0};
                ci[tc][rt] = acc4{0, 0, 0, 0};
            }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                // column of M that K-step s pairs with lane group g (see tile_row)
                const int kc = 16 * (s >> 2) + tile_row<T>(s & 3, g);
                const int at = 2 * ((16 * rt + n) * W + kc);
                const T ar = (T)(mt * buf[at]), ai = (T)(mt * buf[at + 1]);
                // consecutive products go to different accumulators (2 TC independent chains)
#pragma unroll
                for (int tc = 0; tc < TC; ++tc) {
                    cr[tc][rt] = mfma4(ar, vr[tc][s >> 2][s & 3], cr[tc][rt]);
                    ci[tc][rt] = mfma4(ar, vi[tc][s >> 2][s & 3], ci[tc][rt]);
                }
#pragma unroll
                for (int tc = 0; tc < TC; ++tc) {
                    cr[tc][rt] = mfma4(-ai, vi[tc][s >> 2][s & 3], cr[tc][rt]);
                    ci[tc][rt] = mfma4(ai, vr[tc][s >> 2][s & 3], ci[tc][rt]);
                }
            }
        }
#pragma unroll
        for (int tc = 0; tc < TC; ++tc)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    vr[tc][rt][r] = cr[tc][rt][r];
                    vi[tc][rt][r] = ci[tc][rt][r];
                }
    };
    // at slice k: the diagonal block's column for columns of slice k, zero for columns whose
    // slice is beyond k in the sweep direction (`before`)
    auto fix = [&](int k, bool down) {
#pragma unroll
        for (int tc = 0; tc < TC; ++tc) {
            const bool here = k == l[tc];
            const bool before = down ? k < l[tc] : k > l[tc];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int y = 16 * rt + tile_row<T>(r, g);
                    double2 d = cmk(0.0, 0.0);
                    if (here) d = Gde[(size_t)k * W * W + y * W + y0[tc]];
                    vr[tc][rt][r] = here ? (T)d.x : (before ? (T)0 : vr[tc][rt][r]);
                    vi[tc][rt][r] = here ? (T)d.y : (before ? (T)0 : vi[tc][rt][r]);
                }
        }
    };
    auto store = [&](int k, bool down) {
#pragma unroll
        for (int tc = 0; tc < TC; ++tc) {
            const bool on = valid[tc] && (down ? k >= l[tc] : k < l[tc]);
            if (!on) continue;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int y = 16 * rt + tile_row<T>(r, g);
                    const double xr = vr[tc][rt][r], xi = vi[tc][rt][r];
                    if (STORE_G)
                        Ge[(size_t)(k * W + y) * ldG + col[tc]] = cmk(xr, xi);
                    else
                        Pe[(size_t)(k * W + y) * ldP + col[tc]] = xr * xr + xi * xi;
                }
        }
    };
    // Re v^+ Gamma v per column (Gamma real symmetric): u = Gamma v on the matrix cores, the
    // row sum of Re(conj(v) u) over the four lanes of each column; lane g = 0 gets the result.
    auto quad = [&](int tc) -> double {
        acc4 ur[RT], ui[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            ur[rt] = acc4{0, 0, 0, 0};
            ui[rt] = acc4{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const T a = (T)gme[(16 * rt + n) * W + 16 * (s >> 2) + tile_row<T>(s & 3, g)];
                ur[rt] = mfma4(a, vr[tc][s >> 2][s & 3], ur[rt]);
                ui[rt] = mfma4(a, vi[tc][s >> 2][s & 3], ui[rt]);
            }
        }
        double q = 0.0;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                q = fma((double)vr[tc][rt][r], (double)ur[rt][r],
                        fma((double)vi[tc][rt][r], (double)ui[rt][r], q));
        q += __shfl_xor(q, 16, 64);
        q += __shfl_xor(q, 32, 64);
        return q;
    };

    // ---- downward: k = kmin .. L-1 (gR) -------------------------------------------------
#pragma unroll
    for (int tc = 0; tc < TC; ++tc)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) vr[tc][rt][r] = vi[tc][rt][r] = (T)0;
    stage_block<W, 64 * NW>(Ms, gRe + (size_t)kmin * W * W, tid);
    for (int k = kmin; k < L; ++k) {
        __syncthreads();
        const int b = (k - kmin) & 1;
        if (k + 1 < L)
            stage_block<W, 64 * NW>(Ms + (b ^ 1) * BS, gRe + (size_t)(k + 1) * W * W, tid);
        product(Ms + b * BS);
        fix(k, true);
        store(k, true);
    }
    if (!STORE_G) {
#pragma unroll
        for (int tc = 0; tc < TC; ++tc) {
            const double q = quad(tc);
            if (valid[tc] && g == 0) wR[(size_t)e * N + col[tc]] = q;
            if (valid[tc] && l[tc] == 0) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        cRL[(16 * rt + tile_row<T>(r, g)) * W + y0[tc]] = cmk(vr[tc][rt][r], vi[tc][rt][r]);
            }
        }
    }
    // ---- upward: k = kmax .. 0 (gL) -----------------------------------------------------
#pragma unroll
    for (int tc = 0; tc < TC; ++tc)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) vr[tc][rt][r] = vi[tc][rt][r] = (T)0;
    __syncthreads();
    stage_block<W, 64 * NW>(Ms, gLe + (size_t)kmax * W * W, tid);
    for (int k = kmax; k >= 0; --k) {
        __syncthreads();
        const int b = (kmax - k) & 1;
        if (k > 0) stage_block<W, 64 * NW>(Ms + (b ^ 1) * BS, gLe + (size_t)(k - 1) * W * W, tid);
        product(Ms + b * BS);
        fix(k, false);
        store(k, false);
    }
    if (!STORE_G) {
#pragma unroll
        for (int tc = 0; tc < TC; ++tc) {
            const double q = quad(tc);
            if (valid[tc] && g == 0) wL[(size_t)e * N + col[tc]] = q;
            if (valid[tc] && l[tc] == L - 1) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        cLR[(16 * rt + tile_row<T>(r, g)) * W + y0[tc]] = cmk(vr[tc][rt][r], vi[tc][rt][r]);
            }
        }
    }
}

template <int W, int TC, int NW, bool STORE_G, typename T = double>
static hipError_t launch_fullinv_mfma(const mcnegf_kernel& k, double2* Gc, int64_t ldG,
                                      hipStream_t s) {
    dim3 grid((k.N + 16 * TC * NW - 1) / (16 * TC * NW), k.nE);
    {
        MCNEGF_TIMED(STORE_G ? "fullinv_store_g_kernel" : "fullinv_kernel", s);
        hipLaunchKernelGGL((fullinv_mfma_kernel<W, TC, NW, STORE_G, T>), grid, dim3(64 * NW), 0, s,
                           reinterpret_cast<const double2*>(k.gL),
                           reinterpret_cast<const double2*>(k.gR),
                           reinterpret_cast<const double2*>(k.Gd), k.gam_lead, k.L, k.t, k.p_pitch,
                           k.P, k.wL, k.wR, reinterpret_cast<double2*>(k.corner), Gc, ldG);
    }
    return hipGetLastError();
}

// wavefronts per workgroup sharing one staged block
constexpr int kFullinvWaves16 = 1;
constexpr int kFullinvWaves32 = 4;

template <bool STORE_G>
static hipError_t launch_fullinv_any(const mcnegf_kernel& k, double2* Gc, int64_t ldG,
                                     hipStream_t s) {
    if (k.W == 16) return launch_fullinv_mfma<16, 4, kFullinvWaves16, STORE_G>(k, Gc, ldG, s);
    if (k.W == 32) return launch_fullinv_mfma<32, 2, kFullinvWaves32, STORE_G>(k, Gc, ldG, s);
    switch (k.W) {
#define MCNEGF_CASE(w) \
    case w:            \
        return launch_fullinv_w<w, STORE_G>(k, Gc, ldG, s);
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

hipError_t launch_fullinv(const mcnegf_kernel& k, hipStream_t s) {
    return launch_fullinv_any<false>(k, nullptr, 0, s);
}

// The full inverse with FP32 block products (W = 16 and 32 only; any other width is refused).
hipError_t launch_fullinv_fp32(const mcnegf_kernel& k, hipStream_t s) {
    if (k.W == 16) return launch_fullinv_mfma<16, 4, kFullinvWaves16, false, float>(k, nullptr, 0, s);
    if (k.W == 32) return launch_fullinv_mfma<32, 2, kFullinvWaves32, false, float>(k, nullptr, 0, s);
    return hipErrorInvalidValue;
}

hipError_t launch_fullinv_fp32_store_g(const mcnegf_kernel& k, double2* Gc, int64_t ldG,
                                       hipStream_t s) {
    if (k.W == 16) return launch_fullinv_mfma<16, 4, kFullinvWaves16, true, float>(k, Gc, ldG, s);
    if (k.W == 32) return launch_fullinv_mfma<32, 2, kFullinvWaves32, true, float>(k, Gc, ldG, s);
    return hipErrorInvalidValue;
}

hipError_t launch_fullinv_store_g(const mcnegf_kernel& k, double2* Gc, int64_t ldG,
                                  hipStream_t s) {
    return launch_fullinv_any<true>(k, Gc, ldG, s);
}

}  // namespace mcnegf
