// Random walks of the elastic linear-response Monte Carlo (Sec. II E-F): a walker starts
// in the injection row of lead p (steps 3-4 with the eigen-channel marginalised), then
// repeats step 6' (Eqs. (75), (76)) until a lead is drawn.  The transmission estimator
// Tr Gamma_p A [exit at q] (Eq. (66)) only needs the exit counts, so a walker carries no
// weight: the kernel counts exits at L and R, truncated walks, and sums of steps and squared
// steps per energy.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
// 32x32->64-bit products with multipliers 0xD2511F53, 0xCD9E8D57 and Weyl key increments
// 0x9E3779B9, 0xBB67AE85.  Block j of walker w at energy e has counter (j, w, e, tag) and
// key (seed low, seed high); step n uses words 2(n&1), 2(n&1)+1 of block n>>1 as (a, b):
// bucket c = (a * n) >> 32 with Lemire's rejection of the low word below 2^32 mod n (the
// r-th redraw of step n: word 0 of counter (n, w, e, tag | 2^31), key (key0, key1 ^ r)),
// outcome = b < thr[c] ? c : alias[c].
//
// Execution: persistent wavefronts take chunks of consecutive walker indices of one energy
// from an atomic counter (energy-major, so the tables being read are those of one or two
// energies at a time and stay in L2 / MALL); each lane takes the next walker of the chunk
// as soon as its own walker is absorbed, and every loop iteration performs two steps
// from one Philox block.  Tallies live in registers and are wave-reduced once per chunk.
#include "common.h"

namespace mcnegf {

struct Philox4 {
    uint32_t x[4];
};

__device__ inline Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    Philox4 o;
    o.x[0] = c0;
    o.x[1] = c1;
    o.x[2] = c2;
    o.x[3] = c3;
    return o;
}

struct WalkArgs {
    const uint2* tables;
    int64_t pitch;
    int64_t table_stride;  // entries per energy
    uint32_t n_out, N;
    uint32_t nE;
    uint32_t key0, key1, tag;
    uint32_t wbegin, wend;  // walker index range [wbegin, wend)
    uint32_t chunk, chunks_per_energy;
    uint32_t max_steps;
    uint32_t* counter;
    int64_t* tallies;
    uint32_t* status;
};

__device__ inline uint32_t lemire_redraw(uint32_t a, uint32_t n_out, uint32_t step, uint32_t w,
                                         uint32_t e, const WalkArgs& A) {
    const uint32_t thresh = (0u - n_out) % n_out;
    uint32_t r = 0;
    for (;;) {
        const uint64_t m = (uint64_t)a * n_out;
        if ((uint32_t)m >= thresh) return (uint32_t)(m >> 32);
        ++r;
        a = philox4x32_10(step, w, e, A.tag | 0x80000000u, A.key0, A.key1 ^ r).x[0];
    }
}

__global__ void __launch_bounds__(256) walk_kernel(WalkArgs A) {
    const int lane = threadIdx.x & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t total_chunks = A.nE * A.chunks_per_energy;
    const uint32_t n_out = A.n_out;
    const uint32_t N = A.N;
    const uint32_t inject_row = N + (A.tag & 1u);
    for (;;) {
        uint32_t ch = 0;
        if (lane == 0) ch = atomicAdd(A.counter, 1u);
        ch = __builtin_amdgcn_readfirstlane(ch);
        if (ch >= total_chunks) break;
        const uint32_t e = ch / A.chunks_per_energy;
        const uint32_t w0 = A.wbegin + (ch - e * A.chunks_per_energy) * A.chunk;
        const uint32_t w1 = min(w0 + A.chunk, A.wend);
        const uint2* tab = A.tables + (size_t)e * A.table_stride;
        uint32_t next = w0;
        bool active = false;
        uint32_t w = 0, s = 0, n = 0;
        uint32_t cL = 0, cR = 0, tr = 0;
        uint64_t s1 = 0, s2 = 0;
        for (;;) {
            const uint64_t need = __ballot(!active);
            if (need) {
                const uint32_t avail = w1 - next;
                const uint32_t before = __popcll(need & lt_mask);
                if (!active && before < avail) {
                    w = next + before;
                    s = inject_row;
                    n = 0;
                    active = true;
                }
                const uint32_t cnt = __popcll(need);
                next += cnt < avail ? cnt : avail;
            }
            if (__ballot(active) == 0ull) break;
            if (active) {
                const Philox4 x = philox4x32_10(n >> 1, w, e, A.tag, A.key0, A.key1);
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    if (active) {
                        const uint32_t a = x.x[2 * half], b = x.x[2 * half + 1];
                        const uint64_t m = (uint64_t)a * n_out;
                        uint32_t c = (uint32_t)(m >> 32);
                        if ((uint32_t)m < n_out) c = lemire_redraw(a, n_out, n, w, e, A);
                        const uint2 ent = tab[(size_t)s * A.pitch + c];
                        const uint32_t nxt = (b < ent.x) ? c : ent.y;
                        ++n;
                        if (nxt >= N) {
                            if (nxt == N) ++cL; else ++cR;
                            s1 += n;
                            s2 += (uint64_t)n * n;
                            active = false;
                        } else if (n >= A.max_steps) {
                            ++tr;
                            s1 += n;
                            s2 += (uint64_t)n * n;
                            active = false;
                        } else {
                            s = nxt;
                        }
                    }
                }
            }
        }
        // wave reduction of the chunk's tallies
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            cL += __shfl_xor(cL, off, 64);
            cR += __shfl_xor(cR, off, 64);
            tr += __shfl_xor(tr, off, 64);
            s1 += __shfl_xor(s1, off, 64);
            s2 += __shfl_xor(s2, off, 64);
        }
        if (lane == 0) {
            unsigned long long* t =
                reinterpret_cast<unsigned long long*>(A.tallies + (size_t)e * MCNEGF_TALLY_N);
            atomicAdd(t + MCNEGF_TALLY_EXIT_L, (unsigned long long)cL);
            atomicAdd(t + MCNEGF_TALLY_EXIT_R, (unsigned long long)cR);
            if (tr) {
                atomicAdd(t + MCNEGF_TALLY_TRUNC, (unsigned long long)tr);
                atomicOr(A.status, MCNEGF_FLAG_TRUNC);
            }
            atomicAdd(t + MCNEGF_TALLY_STEPS, (unsigned long long)s1);
            atomicAdd(t + MCNEGF_TALLY_STEPS2, (unsigned long long)s2);
        }
    }
}

__global__ void reset_counter_kernel(uint32_t* counter) { counter[0] = 0u; }

hipError_t launch_walk(const mcnegf_kernel& k, uint64_t seed, uint32_t tag, uint32_t walker_begin,
                       uint32_t n_walkers, uint32_t max_steps, int64_t* tallies, hipStream_t s) {
    WalkArgs A;
    A.tables = reinterpret_cast<const uint2*>(k.alias);
    A.pitch = k.alias_pitch;
    A.table_stride = (int64_t)k.n_out * k.alias_pitch;
    A.n_out = (uint32_t)k.n_out;
    A.N = (uint32_t)k.N;
    A.nE = (uint32_t)k.nE;
    A.key0 = (uint32_t)(seed & 0xffffffffu);
    A.key1 = (uint32_t)(seed >> 32);
    A.tag = tag;
    A.wbegin = walker_begin;
    A.wend = walker_begin + n_walkers;
    // chunk: about two chunks per wavefront of a full grid, 64..4096 walkers
    const uint64_t total = (uint64_t)n_walkers * (uint64_t)k.nE;
    const int blocks = 2048;  // 8192 wavefronts of 64 lanes
    uint64_t ch = total / ((uint64_t)blocks * 4 * 2);
    ch = ch < 64 ? 64 : (ch > 4096 ? 4096 : ch);
    ch = (ch + 63) / 64 * 64;
    A.chunk = (uint32_t)ch;
    A.chunks_per_energy = (uint32_t)((n_walkers + ch - 1) / ch);
    A.max_steps = max_steps;
    A.counter = k.counters;
    A.tallies = tallies;
    A.status = k.status;
    {
        MCNEGF_TIMED("reset_counter_kernel", s);
        hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, k.counters);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const uint64_t waves_needed = (uint64_t)A.nE * A.chunks_per_energy;
    const uint64_t nb = (waves_needed + 3) / 4;
    {
        MCNEGF_TIMED("walk_kernel", s);
        hipLaunchKernelGGL(walk_kernel, dim3((unsigned)(nb < (uint64_t)blocks ? nb : blocks)),
                           dim3(256), 0, s, A);
    }
    return hipGetLastError();
}

}  // namespace mcnegf
