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
// in grid-stride order (chunk ids are energy-major, so the wavefronts of the grid work on a
// window of a few energies at a time whose tables stay in L2 / MALL); each lane takes the
// next walker of its chunk as soon as its own walker is absorbed, and every loop iteration
// performs two steps from one Philox block.
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
    uint32_t nE;      // energies in this launch
    uint32_t e_off;   // index of the first of them (the Philox counter uses e_off + e)
    uint32_t key0, key1, tag;
    uint32_t wbegin, wend;  // walker index range [wbegin, wend)
    uint32_t chunk, chunks_per_energy;
    uint32_t max_steps;
    int64_t* tallies;
    uint32_t* status;
};

// Every branch in the loops below is wave-uniform (its condition is a ballot or a value
// computed identically in all lanes), and per-lane differences are expressed as selects:
// the compiler does not guarantee that lanes which took a divergent branch rejoin the others
// before a later cross-lane operation (ballot, shuffle, readfirstlane) in the same loop, so
// the walker keeps the whole wavefront active at every one of them.  Tallies go to LDS
// (every lane adds its own counts) and reach global memory once, after all loops.
struct Step {
    uint32_t s, n;
    bool active;
};

// One transition draw for every lane of the wavefront; lanes with !st.active compute and
// discard.  (a, b) are the step's two Philox words; counts are added for lanes whose walk
// ends here.
__device__ inline void walk_step(Step& st, uint32_t w, uint32_t e, uint32_t a, uint32_t b,
                                 const uint2* __restrict__ tab, const WalkArgs& A,
                                 uint32_t& cL, uint32_t& cR, uint32_t& tr, uint64_t& s1,
                                 uint64_t& s2) {
    const uint32_t n_out = A.n_out;
    uint64_t m = (uint64_t)a * n_out;
    uint32_t thresh = (0u - n_out) % n_out;
    bool rej = st.active && ((uint32_t)m < thresh);
    uint32_t r = 0;
    while (__ballot(rej) != 0ull) {  // rare (probability < n / 2^32 per step); uniform loop
        ++r;
        const uint32_t a2 =
            philox4x32_10(st.n, w, e, A.tag | 0x80000000u, A.key0, A.key1 ^ r).x[0];
        const uint64_t m2 = (uint64_t)a2 * n_out;
        m = rej ? m2 : m;
        rej = rej && ((uint32_t)m2 < thresh);
    }
    const uint32_t c = (uint32_t)(m >> 32);
    const uint2 ent = tab[(size_t)st.s * A.pitch + c];
    const uint32_t nxt = (b < ent.x) ? c : ent.y;
    const uint32_t n1 = st.n + 1;
    const bool absorbed = st.active && nxt >= A.N;
    const bool trunc = st.active && !absorbed && n1 >= A.max_steps;
    const bool ends = absorbed || trunc;
    cL += (absorbed && nxt == A.N) ? 1u : 0u;
    cR += (absorbed && nxt != A.N) ? 1u : 0u;
    tr += trunc ? 1u : 0u;
    s1 += ends ? (uint64_t)n1 : 0ull;
    s2 += ends ? (uint64_t)n1 * n1 : 0ull;
    st.s = (st.active && !ends) ? nxt : st.s;
    st.n = st.active ? n1 : st.n;
    st.active = st.active && !ends;
}

__global__ void __launch_bounds__(256) walk_kernel(WalkArgs A) {
    extern __shared__ unsigned long long lds_tally[];  // [nE][5]
    const int lane = threadIdx.x & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t nE = A.nE;
    for (uint32_t i = threadIdx.x; i < nE * MCNEGF_TALLY_N; i += blockDim.x) lds_tally[i] = 0ull;
    __syncthreads();
    const uint32_t total_chunks = nE * A.chunks_per_energy;
    const uint32_t waves = __builtin_amdgcn_readfirstlane(gridDim.x * (blockDim.x >> 6));
    const uint32_t wave_id =
        __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const uint32_t inject_row = A.N + (A.tag & 1u);
    uint32_t trunc_any = 0;
    for (uint32_t ch = wave_id; ch < total_chunks; ch += waves) {
        const uint32_t el = ch / A.chunks_per_energy;  // energy within this launch
        const uint32_t e = A.e_off + el;                 // energy index of the streams
        const uint32_t w0 = A.wbegin + (ch - el * A.chunks_per_energy) * A.chunk;
        const uint32_t w1 = min(w0 + A.chunk, A.wend);
        const uint2* tab = A.tables + (size_t)el * A.table_stride;
        uint32_t next = w0;
        Step st = {inject_row, 0u, false};
        uint32_t w = 0;
        uint32_t cL = 0, cR = 0, tr = 0;
        uint64_t s1 = 0, s2 = 0;
        for (;;) {
            // refill: idle lanes take the next walker indices of the chunk, in lane order
            const uint64_t need = __ballot(!st.active);
            const uint32_t avail = w1 - next;
            const uint32_t before = __popcll(need & lt_mask);
            const bool take = !st.active && before < avail;
            w = take ? next + before : w;
            st.s = take ? inject_row : st.s;
            st.n = take ? 0u : st.n;
            st.active = st.active || take;
            const uint32_t cnt = __popcll(need);
            next += cnt < avail ? cnt : avail;
            if (__ballot(st.active) == 0ull) break;
            // two steps from one Philox block (step n uses words 2(n&1), 2(n&1)+1 of block n>>1;
            // active walkers enter the iteration at even n)
            const Philox4 x = philox4x32_10(st.n >> 1, w, e, A.tag, A.key0, A.key1);
            walk_step(st, w, e, x.x[0], x.x[1], tab, A, cL, cR, tr, s1, s2);
            walk_step(st, w, e, x.x[2], x.x[3], tab, A, cL, cR, tr, s1, s2);
        }
        unsigned long long* t = lds_tally + (size_t)el * MCNEGF_TALLY_N;
        atomicAdd(t + MCNEGF_TALLY_EXIT_L, (unsigned long long)cL);
        atomicAdd(t + MCNEGF_TALLY_EXIT_R, (unsigned long long)cR);
        atomicAdd(t + MCNEGF_TALLY_TRUNC, (unsigned long long)tr);
        atomicAdd(t + MCNEGF_TALLY_STEPS, (unsigned long long)s1);
        atomicAdd(t + MCNEGF_TALLY_STEPS2, (unsigned long long)s2);
        trunc_any |= tr;
    }
    __syncthreads();
    unsigned long long* gt = reinterpret_cast<unsigned long long*>(A.tallies);
    for (uint32_t i = threadIdx.x; i < nE * MCNEGF_TALLY_N; i += blockDim.x) {
        const unsigned long long v = lds_tally[i];
        if (v) atomicAdd(gt + i, v);
    }
    if (trunc_any) atomicOr(A.status, MCNEGF_FLAG_TRUNC);
}

hipError_t launch_walk(const mcnegf_kernel& k, uint64_t seed, uint32_t tag, uint32_t walker_begin,
                       uint32_t n_walkers, uint32_t max_steps, int64_t* tallies, hipStream_t s) {
    // energies per launch: the LDS tallies ([energies][5] int64) must fit the 160 KB of a CU
    constexpr uint32_t kMaxEnergiesPerLaunch = 2048;
    const size_t max_lds = (size_t)kMaxEnergiesPerLaunch * MCNEGF_TALLY_N * 8;
    hipError_t err = hipFuncSetAttribute((const void*)walk_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds);
    if (err != hipSuccess) return err;
    for (uint32_t e_off = 0; e_off < (uint32_t)k.nE; e_off += kMaxEnergiesPerLaunch) {
        WalkArgs A;
        const uint32_t nE = min((uint32_t)k.nE - e_off, kMaxEnergiesPerLaunch);
        A.table_stride = (int64_t)k.n_out * k.alias_pitch;
        A.tables = reinterpret_cast<const uint2*>(k.alias) + (size_t)e_off * A.table_stride;
        A.pitch = k.alias_pitch;
        A.n_out = (uint32_t)k.n_out;
        A.N = (uint32_t)k.N;
        A.nE = nE;
        A.e_off = e_off;
        A.key0 = (uint32_t)(seed & 0xffffffffu);
        A.key1 = (uint32_t)(seed >> 32);
        A.tag = tag;
        A.wbegin = walker_begin;
        A.wend = walker_begin + n_walkers;
        // chunk: about four chunks per wavefront of a full grid, 64..4096 walkers
        const uint64_t total = (uint64_t)n_walkers * nE;
        const int max_blocks = 2048;  // 8192 wavefronts of 64 lanes
        uint64_t ch = total / ((uint64_t)max_blocks * 4 * 4);
        ch = ch < 64 ? 64 : (ch > 4096 ? 4096 : ch);
        ch = (ch + 63) / 64 * 64;
        A.chunk = (uint32_t)ch;
        A.chunks_per_energy = (uint32_t)((n_walkers + ch - 1) / ch);
        A.max_steps = max_steps;
        A.tallies = tallies + (size_t)e_off * MCNEGF_TALLY_N;
        A.status = k.status;
        const uint64_t waves_needed = (uint64_t)nE * A.chunks_per_energy;
        const uint64_t nb = (waves_needed + 3) / 4;
        const size_t lds = (size_t)nE * MCNEGF_TALLY_N * 8;
        {
            MCNEGF_TIMED("walk_kernel", s);
            hipLaunchKernelGGL(walk_kernel,
                               dim3((unsigned)(nb < (uint64_t)max_blocks ? nb : max_blocks)),
                               dim3(256), lds, s, A);
        }
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    return hipSuccess;
}

}  // namespace mcnegf
