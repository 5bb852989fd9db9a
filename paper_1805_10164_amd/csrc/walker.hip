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
// Execution: persistent wavefronts, one energy group per XCD (see walk_kernel); each lane
// takes the next walker of its wavefront's chunk as soon as its own walker is absorbed, and
// every loop iteration performs two steps from one Philox block.  The keep test compares the
// high 16 bits of b with the bucket's packed entry and reads the low 16 threshold bits only
// on a tie.  A walk's first step reads its injection row from an LDS copy when the launch
// staged one; a finished walk is counted once, when its slot takes the next walker.
#include <algorithm>
#include <mutex>

#include "common.h"

namespace mcnegf {

// Pointer into device global memory; a per-lane pointer chosen by a select keeps its address
// space, so table reads stay global (not flat) loads.
typedef const __attribute__((address_space(1))) uint32_t* gtable_ptr;

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
    const uint32_t* tables;  // packed (thr >> 16) << 16 | alias
    const uint16_t* lows;    // thr & 0xFFFF
    uint32_t pitch32;      // entries per table row (below 2^24)
    int64_t table_stride;  // entries per energy
    uint32_t n_out, N;
    uint32_t nE;      // energies in this launch
    uint32_t e_off;   // index of the first of them (the Philox counter uses e_off + e)
    uint32_t key0, key1, tag;
    uint32_t wbegin, wend;  // walker index range [wbegin, wend)
    uint32_t chunk, chunks_per_energy;
    uint32_t groups;  // energy groups: energy el belongs to group el % groups
    uint32_t max_steps;
    uint32_t stage_inject;  // 1: each workgroup copies its energies' injection rows into LDS
    int64_t* tallies;
    uint32_t* status;
};

// One unit of a batched walk: one energy of one built kernel.
struct WalkUnit {
    const uint32_t* tables;  // this energy's packed alias rows
    const uint16_t* lows;
    int64_t* tally;          // this energy's [5] tallies
    uint32_t* status;        // the kernel's status word
    const uint32_t* ids;     // with per-unit counts: the unit's walker indices (else null)
    uint32_t pitch, n_out, N, e, tag, nw;  // nw: the unit's walker count (per-unit mode)
};

struct WalkBatchArgs {
    const WalkUnit* units;
    uint32_t n_units;
    uint32_t key0, key1;
    uint32_t wbegin, wend;
    uint32_t chunk, chunks_per_unit;
    uint32_t groups;
    uint32_t max_steps;
    int64_t* tally_override;  // non-null: unit u's counts go to tally_override[u][5]
    // Per-unit counts (energy-sampled walks): chunk_start[u] = first chunk of unit u
    // ([n_units + 1], device); unit u walks U.ids[0 .. U.nw) in chunks of `chunk`.  Null:
    // every unit walks [wbegin, wend).
    const uint32_t* chunk_start;
};

// Every branch in the loops below that encloses a cross-lane operation is wave-uniform (its
// condition is a ballot or a value computed identically in all lanes), and per-lane
// differences are expressed as selects: the compiler does not guarantee that lanes which took
// a divergent branch rejoin the others before a later cross-lane operation (ballot, shuffle,
// readfirstlane) in the same loop, so the walker keeps the whole wavefront active at every
// one of them.  The only divergent regions hold a table load or LDS atomics.
struct Step {
    uint32_t s, n;
    bool active;
};

struct Tally {
    uint32_t cL, cR, tr;
    uint64_t s1, s2;
};

// One transition draw for each of the K walker slots of every lane; inactive slots compute and
// discard.  (a[k], b[k]) are slot k's two Philox words for this step; tb[k] is the first
// packed entry of slot k's energy.  The K table loads are independent and issued together, so
// a wavefront keeps K memory requests in flight per lane.  A walk that ends leaves its exit
// state in s (lead L = N, lead R = N + 1, a probe when truncated) and its step count in n; it
// is counted when its slot is refilled (count_ended), not here.
template <int K>
__device__ inline void walk_steps(Step (&st)[K], const gtable_ptr (&tb)[K],
                                  const uint32_t (&w)[K], const uint32_t (&el)[K],
                                  const uint32_t (&lq)[K], const uint32_t* lds_inj,
                                  const uint32_t (&a)[K], const uint32_t (&b)[K],
                                  const WalkArgs& A) {
    const uint32_t n_out = A.n_out;
    const uint32_t thresh = (0u - n_out) % n_out;
    uint64_t m[K];
    bool rej[K];
    uint64_t rb = 0ull;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        m[k] = (uint64_t)a[k] * n_out;
        rej[k] = st[k].active && ((uint32_t)m[k] < thresh);
        rb |= __ballot(rej[k]);
    }
    uint32_t r = 0;
    while (rb != 0ull) {  // rare (probability < n / 2^32 per step); uniform loop
        ++r;
        rb = 0ull;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t a2 = philox4x32_10(st[k].n, w[k], A.e_off + el[k],
                                              A.tag | 0x80000000u, A.key0, A.key1 ^ r).x[0];
            const uint64_t m2 = (uint64_t)a2 * n_out;
            m[k] = rej[k] ? m2 : m[k];
            rej[k] = rej[k] && ((uint32_t)m2 < thresh);
            rb |= __ballot(rej[k]);
        }
    }
    // entry offset within the energy's table: row * pitch + bucket, both below 2^24 and the
    // sum below 2^32 (at most 16320 rows of pitch 16320)
    // Only active slots read: a walk's first step (n = 0, the injection row) from the copy of
    // that row in LDS when the launch staged it, every other step from the table in memory.
    // The two kinds of read go to separate registers (one register for both would make the
    // second wait for the first) and are merged by a select once all K are issued.
    uint32_t c[K], off[K], ent[K], eg[K], el_[K];
    bool inj[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        c[k] = (uint32_t)(m[k] >> 32);
        off[k] = __umul24(st[k].s, A.pitch32) + c[k];
        inj[k] = A.stage_inject && st[k].n == 0u;
        eg[k] = 0u;
        el_[k] = 0u;
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (st[k].active && !inj[k]) eg[k] = tb[k][off[k]];
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (st[k].active && inj[k]) el_[k] = lds_inj[lq[k] + c[k]];
#pragma unroll
    for (int k = 0; k < K; ++k) ent[k] = inj[k] ? el_[k] : eg[k];
    bool keep[K], tie[K];
    uint64_t tb_any = 0ull;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        // high 16 threshold bits: b keeps the bucket below them, ties read the low 16 bits
        keep[k] = b[k] < (ent[k] & ~kAliasIdxMask);
        tie[k] = st[k].active && ((b[k] ^ ent[k]) >> kAliasIdxBits) == 0u;
        tb_any |= __ballot(tie[k]);
    }
    if (tb_any != 0ull) {  // rare (probability 2^-16 per lane and step); uniform branch
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t lo =
                tie[k] ? (uint32_t)A.lows[(size_t)el[k] * A.table_stride + off[k]] : 0u;
            keep[k] = tie[k] ? (b[k] & kAliasIdxMask) < lo : keep[k];
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t nxt = keep[k] ? c[k] : (ent[k] & kAliasIdxMask);
        const uint32_t n1 = st[k].n + 1;
        const bool active = st[k].active;
        // absorbed at a lead (nxt >= N) or truncated at max_steps
        const bool ends = nxt >= A.N || n1 >= A.max_steps;
        st[k].s = active ? nxt : st[k].s;
        st[k].n = active ? n1 : st[k].n;
        st[k].active = active && !ends;
    }
}

// Adds the walk that ended in a slot (done: the slot holds one that is not counted yet) to
// counts: exit by its final state (lead L = N, lead R = N + 1, a probe when truncated), its
// step count and squared step count.
__device__ inline void count_ended_lane(uint32_t& cL, uint32_t& cR, uint32_t& tr, uint64_t& s1,
                                        uint64_t& s2, bool done, const Step& s, uint32_t N) {
    const uint64_t n = done ? (uint64_t)s.n : 0ull;
    cL += (done && s.s == N) ? 1u : 0u;
    cR += (done && s.s > N) ? 1u : 0u;
    tr += (done && s.s < N) ? 1u : 0u;
    s1 += n;
    s2 += n * n;
}
// The same into a slot's counts (the per-kernel walker's slots move between energies).
__device__ inline void count_ended(Tally& t, bool done, const Step& s, uint32_t N) {
    count_ended_lane(t.cL, t.cR, t.tr, t.s1, t.s2, done, s, N);
}

// Adds a slot's counts for energy el to the block's LDS tallies (per-lane; called in
// divergent code, no cross-lane operation inside).
__device__ inline void tally_flush(unsigned long long* lds_tally, uint32_t el, const Tally& t) {
    unsigned long long* p = lds_tally + (size_t)el * MCNEGF_TALLY_N;
    if (t.cL) atomicAdd(p + MCNEGF_TALLY_EXIT_L, (unsigned long long)t.cL);
    if (t.cR) atomicAdd(p + MCNEGF_TALLY_EXIT_R, (unsigned long long)t.cR);
    if (t.tr) atomicAdd(p + MCNEGF_TALLY_TRUNC, (unsigned long long)t.tr);
    if (t.s1) atomicAdd(p + MCNEGF_TALLY_STEPS, (unsigned long long)t.s1);
    if (t.s2) atomicAdd(p + MCNEGF_TALLY_STEPS2, (unsigned long long)t.s2);
}

// Work layout.  Energy el belongs to group el % groups and workgroup b to group b % groups;
// consecutive workgroups are dispatched to the 8 XCDs in turn, so with 8 groups all walkers of
// an energy run on one XCD, whose L2 then holds that energy's table.  A group's work is the
// energy-major list of chunks (chunk c of its q-th energy has id q * chunks_per_energy + c);
// its wavefronts take ids in stride order, and with one chunk per wavefront and energy the
// wavefronts of a group walk one energy at a time.  Every lane runs K walker slots.  A slot
// whose walk has ended takes the next walker index of the wavefront's current chunk, moving
// on to the wavefront's next chunk (the next energy) when the current one is used up, so no
// slot waits for the slowest walk of a chunk; a slot's counts are kept in registers for its
// current energy and added to LDS when it changes energy.
template <int K>
__global__ void __launch_bounds__(256) walk_kernel(WalkArgs A) {
    // LDS: tallies [nE][5], then (stage_inject) the injection row of each of the group's
    // energies, [nq][n_out] packed entries
    extern __shared__ unsigned long long lds_tally[];
    uint32_t* lds_inj = reinterpret_cast<uint32_t*>(lds_tally + (size_t)A.nE * MCNEGF_TALLY_N);
    const int lane = threadIdx.x & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t nE = A.nE;
    const uint32_t G = A.groups;
    const uint32_t grp = blockIdx.x % G;
    const uint32_t nq = (nE - grp + G - 1) / G;  // energies of this group
    const uint32_t inject_row = A.N + (A.tag & 1u);
    for (uint32_t i = threadIdx.x; i < nE * MCNEGF_TALLY_N; i += blockDim.x) lds_tally[i] = 0ull;
    if (A.stage_inject) {
        for (uint32_t q = 0; q < nq; ++q) {
            const uint32_t* row = A.tables + (size_t)(grp + q * G) * A.table_stride +
                                  (size_t)inject_row * A.pitch32;
            for (uint32_t i = threadIdx.x; i < A.n_out; i += blockDim.x)
                lds_inj[q * A.n_out + i] = row[i];
        }
    }
    __syncthreads();
    const uint32_t wpb = blockDim.x >> 6;
    const uint32_t waves = __builtin_amdgcn_readfirstlane((gridDim.x / G) * wpb);
    const uint32_t lw =
        __builtin_amdgcn_readfirstlane((blockIdx.x / G) * wpb + (threadIdx.x >> 6));
    const uint32_t total = nq * A.chunks_per_energy;

    // the wavefront's cursor: chunk id, its energy, next walker index and end
    uint32_t cid = lw, cel = 0, clq = 0, next = 0, wend = 0;
    auto open_chunk = [&](uint32_t id) {
        const uint32_t q = id / A.chunks_per_energy;
        cel = grp + q * G;
        clq = q * A.n_out;
        next = A.wbegin + (id - q * A.chunks_per_energy) * A.chunk;
        wend = (uint32_t)min((uint64_t)next + A.chunk, (uint64_t)A.wend);
    };
    if (cid < total) open_chunk(cid);

    Step st[K];
    uint32_t w[K], el[K], tel[K];  // walker index, its energy, energy of the counts in t
    gtable_ptr tb[K];              // the packed table of energy el
    uint32_t lq[K];                // the LDS offset of energy el's injection row
    Tally t[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        st[k] = Step{inject_row, 0u, false};
        w[k] = el[k] = tel[k] = lq[k] = 0u;
        tb[k] = (gtable_ptr)A.tables;
        t[k] = Tally{0u, 0u, 0u, 0ull, 0ull};
    }
    uint32_t trunc_any = 0;
    for (;;) {
        // refill idle slots (slot-major, then lane order) from the cursor's chunks
        while (cid < total) {
            uint64_t need[K];
            uint32_t tot = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                need[k] = __ballot(!st[k].active);
                tot += __popcll(need[k]);
            }
            if (tot == 0) break;
            const uint32_t avail = wend - next;
            uint32_t base = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t before = base + __popcll(need[k] & lt_mask);
                const bool take = !st[k].active && before < avail;
                // the walk this slot finished (a slot that never walked has n = 0) is counted
                // for its energy el[k] == tel[k] before the slot moves on
                count_ended(t[k], take && st[k].n != 0u, st[k], A.N);
                const bool flush = take && cel != tel[k];
                if (__ballot(flush) != 0ull) {
                    trunc_any |= flush ? t[k].tr : 0u;
                    if (flush) tally_flush(lds_tally, tel[k], t[k]);
                    t[k].cL = flush ? 0u : t[k].cL;
                    t[k].cR = flush ? 0u : t[k].cR;
                    t[k].tr = flush ? 0u : t[k].tr;
                    t[k].s1 = flush ? 0ull : t[k].s1;
                    t[k].s2 = flush ? 0ull : t[k].s2;
                    tel[k] = flush ? cel : tel[k];
                }
                w[k] = take ? next + before : w[k];
                el[k] = take ? cel : el[k];
                lq[k] = take ? clq : lq[k];
                tb[k] = take ? (gtable_ptr)(A.tables + (size_t)cel * A.table_stride) : tb[k];
                st[k].s = take ? inject_row : st[k].s;
                st[k].n = take ? 0u : st[k].n;
                st[k].active = st[k].active || take;
                base += __popcll(need[k]);
            }
            next += tot < avail ? tot : avail;
            if (next >= wend) {
                cid += waves;
                if (cid < total) open_chunk(cid);
            }
        }
        uint64_t any = 0ull;
#pragma unroll
        for (int k = 0; k < K; ++k) any |= __ballot(st[k].active);
        if (any == 0ull) break;
        // two steps from one Philox block per slot (step n uses words 2(n&1), 2(n&1)+1 of
        // block n>>1; active walkers enter the iteration at even n)
        uint32_t a0[K], b0[K], a1[K], b1[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const Philox4 x =
                philox4x32_10(st[k].n >> 1, w[k], A.e_off + el[k], A.tag, A.key0, A.key1);
            a0[k] = x.x[0];
            b0[k] = x.x[1];
            a1[k] = x.x[2];
            b1[k] = x.x[3];
        }
        walk_steps<K>(st, tb, w, el, lq, lds_inj, a0, b0, A);
        walk_steps<K>(st, tb, w, el, lq, lds_inj, a1, b1, A);
    }
    // walks that ended after their slot's last refill
#pragma unroll
    for (int k = 0; k < K; ++k) {
        count_ended(t[k], st[k].n != 0u, st[k], A.N);
        trunc_any |= t[k].tr;
        tally_flush(lds_tally, tel[k], t[k]);
    }
    __syncthreads();
    unsigned long long* gt = reinterpret_cast<unsigned long long*>(A.tallies);
    for (uint32_t i = threadIdx.x; i < nE * MCNEGF_TALLY_N; i += blockDim.x) {
        const unsigned long long v = lds_tally[i];
        if (v) atomicAdd(gt + i, v);
    }
    if (trunc_any) atomicOr(A.status, MCNEGF_FLAG_TRUNC);
}

constexpr int kWalkSlots = 3;

hipError_t launch_walk(const mcnegf_kernel& k, uint64_t seed, uint32_t tag, uint32_t walker_begin,
                       uint32_t n_walkers, uint32_t max_steps, int64_t* tallies, hipStream_t s) {
    if (n_walkers == 0) return hipSuccess;
    // One launch per round of kXcds * kEnergiesPerXcd energies: a kernel boundary keeps the
    // wavefronts of an XCD on the same energies, whose tables then stay in that XCD's L2
    // (without it, wavefronts drift apart over many energies and the L2 thrashes).  Fewer than
    // kXcds energies go in one launch in a single group.
    constexpr uint32_t kXcds = 8;
    constexpr uint32_t kEnergiesPerXcd = 4;
    constexpr uint32_t kMaxEnergiesPerLaunch = kXcds * kEnergiesPerXcd;
    const void* fn = (const void*)walk_kernel<kWalkSlots>;
    int dev = 0, cus = 0;
    hipError_t err;
    if ((err = hipGetDevice(&dev)) != hipSuccess) return err;
    if ((err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
        hipSuccess)
        return err;
    // A workgroup copies the injection rows of its group's energies into LDS (a walk's first
    // step then reads LDS, not memory) while they take at most kInjectLdsBytes.
    constexpr size_t kInjectLdsBytes = 32768;
    const size_t lds = (size_t)kMaxEnergiesPerLaunch * MCNEGF_TALLY_N * 8 + kInjectLdsBytes;
    // persistent grid: no more workgroups than can be resident at once
    int per_cu = 0;
    if ((err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds)) != hipSuccess)
        return err;
    const uint32_t max_blocks = (uint32_t)(per_cu < 1 ? 1 : per_cu) * (uint32_t)cus;
    for (uint32_t e_off = 0; e_off < (uint32_t)k.nE; e_off += kMaxEnergiesPerLaunch) {
        WalkArgs A;
        const uint32_t nE = min((uint32_t)k.nE - e_off, kMaxEnergiesPerLaunch);
        A.table_stride = (int64_t)k.n_out * k.alias_pitch;
        A.tables = k.alias + (size_t)e_off * A.table_stride;
        A.lows = k.alias_lo + (size_t)e_off * A.table_stride;
        A.pitch32 = (uint32_t)k.alias_pitch;
        A.n_out = (uint32_t)k.n_out;
        A.N = (uint32_t)k.N;
        A.nE = nE;
        A.e_off = e_off;
        A.key0 = (uint32_t)(seed & 0xffffffffu);
        A.key1 = (uint32_t)(seed >> 32);
        A.tag = tag;
        A.wbegin = walker_begin;
        A.wend = walker_begin + n_walkers;
        A.groups = nE >= kXcds ? kXcds : 1u;
        // wavefronts per group: at most the grid's share, and about two walkers per slot
        const uint64_t nq = (nE + A.groups - 1) / A.groups;
        const uint64_t walkers_per_group = nq * n_walkers;
        uint64_t wg = walkers_per_group / (64ull * kWalkSlots * 2);
        uint64_t wg_max = (uint64_t)max_blocks / A.groups * 4;
        wg_max = wg_max < 4 ? 4 : wg_max;
        wg = wg < 4 ? 4 : (wg > wg_max ? wg_max : wg);
        const uint64_t bpg = (wg + 3) / 4;
        // one chunk per wavefront and energy
        const uint64_t ch = (n_walkers + bpg * 4 - 1) / (bpg * 4);
        A.chunk = (uint32_t)ch;
        A.chunks_per_energy = (uint32_t)((n_walkers + ch - 1) / ch);
        A.max_steps = max_steps;
        A.tallies = tallies + (size_t)e_off * MCNEGF_TALLY_N;
        A.status = k.status;
        const size_t inj_bytes = (size_t)nq * (size_t)k.n_out * 4;
        A.stage_inject = inj_bytes <= kInjectLdsBytes ? 1u : 0u;
        const size_t lds_launch =
            (size_t)nE * MCNEGF_TALLY_N * 8 + (A.stage_inject ? inj_bytes : 0);
        {
            MCNEGF_TIMED("walk_kernel", s);
            hipLaunchKernelGGL(walk_kernel<kWalkSlots>, dim3((unsigned)(bpg * A.groups)),
                               dim3(256), lds_launch, s, A);
        }
        if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    return hipSuccess;
}

// ---- batched walk over many built kernels (systems of different sizes, all energies) ------
//
// Work list: units u = (kernel, energy), each with the same walker index range, cut into
// chunks of `chunk` walkers.  Unit u belongs to group u % groups and workgroup b to group
// b % groups (with 8 groups, each XCD walks its own units); a group's wavefronts take its
// chunks in stride order.  A wavefront walks one chunk at a time, so the unit's table, sizes
// and Philox tag are wave-uniform; its K slots per lane refill from the chunk until it is used
// up, and when every slot has finished the chunk's counts are reduced across the wavefront and
// added to the unit's tallies with one atomic per slot of the tally.  A walker's path depends
// only on (seed, step, walker, energy, tag), so the tallies equal those of mc_negf_walk on each
// kernel for any launch shape.

// A pointer that is the same in every lane, moved to scalar registers.
__device__ inline const void* uniform_ptr(const void* p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const void*)(((uint64_t)hi << 32) | lo);
}

// 64-bit sum over the wavefront (every lane gets it); all lanes active.
__device__ inline uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int K>
__global__ void walk_batch_kernel(WalkBatchArgs A) {
    const int lane = threadIdx.x & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t G = A.groups;
    const uint32_t grp = blockIdx.x % G;
    const uint32_t wpb = blockDim.x >> 6;
    const uint32_t waves = __builtin_amdgcn_readfirstlane((gridDim.x / G) * wpb);
    const uint32_t lw =
        __builtin_amdgcn_readfirstlane((blockIdx.x / G) * wpb + (threadIdx.x >> 6));
    const uint32_t nq = (A.n_units > grp) ? (A.n_units - grp + G - 1) / G : 0u;  // units of the group
    const bool per_unit = A.chunk_start != nullptr;  // (then G == 1)
    const uint32_t total = per_unit ? A.chunk_start[A.n_units] : nq * A.chunks_per_unit;
    uint32_t trunc_any = 0;
    for (uint32_t cid0 = lw; cid0 < total; cid0 += waves) {  // uniform loop
        const uint32_t cid = __builtin_amdgcn_readfirstlane(cid0);
        uint32_t q, u;
        if (per_unit) {  // last unit whose first chunk is <= cid (uniform binary search)
            uint32_t lo = 0, hi = A.n_units;
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (A.chunk_start[mid] <= cid) lo = mid; else hi = mid;
            }
            u = __builtin_amdgcn_readfirstlane(lo);
            q = 0;
        } else {
            q = cid / A.chunks_per_unit;
            u = __builtin_amdgcn_readfirstlane(grp + q * G);
        }
        const WalkUnit Uv = A.units[u];
        // the descriptor is the same in every lane: keep its fields in scalar registers
        WalkUnit U;
        U.tables = (const uint32_t*)uniform_ptr(Uv.tables);
        U.lows = (const uint16_t*)uniform_ptr(Uv.lows);
        U.tally = (int64_t*)uniform_ptr(Uv.tally);
        U.status = (uint32_t*)uniform_ptr(Uv.status);
        U.pitch = __builtin_amdgcn_readfirstlane(Uv.pitch);
        U.n_out = __builtin_amdgcn_readfirstlane(Uv.n_out);
        U.N = __builtin_amdgcn_readfirstlane(Uv.N);
        U.e = __builtin_amdgcn_readfirstlane(Uv.e);
        U.tag = __builtin_amdgcn_readfirstlane(Uv.tag);
        U.ids = (const uint32_t*)uniform_ptr(Uv.ids);
        U.nw = __builtin_amdgcn_readfirstlane(Uv.nw);
        // positions [next, wend) of this chunk: walker indices, or indices into U.ids
        uint32_t next, wend;
        if (per_unit) {
            next = (cid - A.chunk_start[u]) * A.chunk;
            wend = (uint32_t)min((uint64_t)next + A.chunk, (uint64_t)U.nw);
        } else {
            next = A.wbegin + (cid - q * A.chunks_per_unit) * A.chunk;
            wend = (uint32_t)min((uint64_t)next + A.chunk, (uint64_t)A.wend);
        }
        const uint32_t n_out = U.n_out, N = U.N;
        const uint32_t thresh = (0u - n_out) % n_out;
        const uint32_t inject_row = N + (U.tag & 1u);
        Step st[K];
        uint32_t w[K];
        uint32_t cL = 0, cR = 0, tr = 0;
        uint64_t s1 = 0, s2 = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            st[k] = Step{inject_row, 0u, false};
            w[k] = 0u;
        }
        for (;;) {
            // refill idle slots (slot-major, then lane order) from the chunk
            if (next < wend) {
                uint64_t need[K];
#pragma unroll
                for (int k = 0; k < K; ++k) need[k] = __ballot(!st[k].active);
                const uint32_t avail = wend - next;
                uint32_t base = 0;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const uint32_t before = base + __popcll(need[k] & lt_mask);
                    const bool take = !st[k].active && before < avail;
                    // the walk this slot finished is counted before the slot takes the next one
                    count_ended_lane(cL, cR, tr, s1, s2, take && st[k].n != 0u, st[k], N);
                    uint32_t wid = next + before;
                    if (U.ids) {  // uniform branch; the load is per lane
                        if (take) wid = U.ids[wid];
                    }
                    w[k] = take ? wid : w[k];
                    st[k].s = take ? inject_row : st[k].s;
                    st[k].n = take ? 0u : st[k].n;
                    st[k].active = st[k].active || take;
                    base += __popcll(need[k]);
                }
                next += base < avail ? base : avail;
            }
            uint64_t any = 0ull;
#pragma unroll
            for (int k = 0; k < K; ++k) any |= __ballot(st[k].active);
            if (any == 0ull) break;
            uint32_t ab[2][2][K];  // [step][word][slot]
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const Philox4 x = philox4x32_10(st[k].n >> 1, w[k], U.e, U.tag, A.key0, A.key1);
                ab[0][0][k] = x.x[0];
                ab[0][1][k] = x.x[1];
                ab[1][0][k] = x.x[2];
                ab[1][1][k] = x.x[3];
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                uint64_t m[K];
                bool rej[K];
                uint64_t rb = 0ull;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    m[k] = (uint64_t)ab[h][0][k] * n_out;
                    rej[k] = st[k].active && ((uint32_t)m[k] < thresh);
                    rb |= __ballot(rej[k]);
                }
                uint32_t r = 0;
                while (rb != 0ull) {  // rare; uniform loop
                    ++r;
                    rb = 0ull;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const uint32_t a2 = philox4x32_10(st[k].n, w[k], U.e, U.tag | 0x80000000u,
                                                          A.key0, A.key1 ^ r).x[0];
                        const uint64_t m2 = (uint64_t)a2 * n_out;
                        m[k] = rej[k] ? m2 : m[k];
                        rej[k] = rej[k] && ((uint32_t)m2 < thresh);
                        rb |= __ballot(rej[k]);
                    }
                }
                // entry offset row * pitch + bucket (both below 2^24, the sum below 2^32); idle
                // slots read nothing
                uint32_t c[K], ent[K], at[K];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    c[k] = (uint32_t)(m[k] >> 32);
                    at[k] = __umul24(st[k].s, U.pitch) + c[k];
                    ent[k] = 0u;
                }
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (st[k].active) ent[k] = U.tables[at[k]];
                bool keep[K], tie[K];
                uint64_t tb = 0ull;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const uint32_t b = ab[h][1][k];
                    keep[k] = (b >> kAliasIdxBits) < (ent[k] >> kAliasIdxBits);
                    tie[k] = st[k].active && (b >> kAliasIdxBits) == (ent[k] >> kAliasIdxBits);
                    tb |= __ballot(tie[k]);
                }
                if (tb != 0ull) {  // rare; uniform branch
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const uint32_t lo = tie[k] ? (uint32_t)U.lows[at[k]] : 0u;
                        keep[k] = tie[k] ? (ab[h][1][k] & kAliasIdxMask) < lo : keep[k];
                    }
                }
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    // a walk that ends keeps its exit state and step count (counted at refill)
                    const uint32_t nxt = keep[k] ? c[k] : (ent[k] & kAliasIdxMask);
                    const uint32_t n1 = st[k].n + 1;
                    const bool active = st[k].active;
                    const bool ends = nxt >= N || n1 >= A.max_steps;
                    st[k].s = active ? nxt : st[k].s;
                    st[k].n = active ? n1 : st[k].n;
                    st[k].active = active && !ends;
                }
            }
        }
        // walks that ended after their slot's last refill
#pragma unroll
        for (int k = 0; k < K; ++k) count_ended_lane(cL, cR, tr, s1, s2, st[k].n != 0u, st[k], N);
        // the chunk is done: one atomic per tally slot for the wavefront
        const uint64_t v0 = wave_sum_u64(cL), v1 = wave_sum_u64(cR), v2 = wave_sum_u64(tr);
        const uint64_t v3 = wave_sum_u64(s1), v4 = wave_sum_u64(s2);
        trunc_any |= (uint32_t)(v2 != 0);
        unsigned long long* gt = reinterpret_cast<unsigned long long*>(
            A.tally_override ? A.tally_override + (size_t)u * MCNEGF_TALLY_N : U.tally);
        if (lane == 0) {
            if (v0) atomicAdd(gt + MCNEGF_TALLY_EXIT_L, (unsigned long long)v0);
            if (v1) atomicAdd(gt + MCNEGF_TALLY_EXIT_R, (unsigned long long)v1);
            if (v2) atomicAdd(gt + MCNEGF_TALLY_TRUNC, (unsigned long long)v2);
            if (v3) atomicAdd(gt + MCNEGF_TALLY_STEPS, (unsigned long long)v3);
            if (v4) atomicAdd(gt + MCNEGF_TALLY_STEPS2, (unsigned long long)v4);
            if (v2 && U.status) atomicOr(U.status, MCNEGF_FLAG_TRUNC);
        }
    }
    (void)trunc_any;
}

size_t walk_unit_bytes() { return sizeof(WalkUnit); }

void fill_walk_unit(void* dst, const mcnegf_kernel& k, int e, uint32_t tag, int64_t* tally) {
    WalkUnit U;
    const size_t stride = (size_t)k.n_out * (size_t)k.alias_pitch;
    U.tables = k.alias + (size_t)e * stride;
    U.lows = k.alias_lo + (size_t)e * stride;
    U.tally = tally + (size_t)e * MCNEGF_TALLY_N;
    U.status = k.status;
    U.pitch = (uint32_t)k.alias_pitch;
    U.n_out = (uint32_t)k.n_out;
    U.N = (uint32_t)k.N;
    U.e = (uint32_t)e;
    U.tag = tag;
    U.ids = nullptr;
    U.nw = 0;
    *static_cast<WalkUnit*>(dst) = U;
}

void fill_walk_unit_ids(void* dst, const mcnegf_kernel& k, int e, uint32_t tag, int64_t* tally,
                        const uint32_t* ids, uint32_t nw) {
    fill_walk_unit(dst, k, e, tag, tally);
    WalkUnit* U = static_cast<WalkUnit*>(dst);
    U->ids = ids;
    U->nw = nw;
}

template <int K>
static hipError_t launch_walk_batch_k(const WalkBatchArgs& A, uint32_t blocks, uint32_t wg,
                                      hipStream_t s) {
    MCNEGF_TIMED("walk_batch_kernel", s);
    hipLaunchKernelGGL(walk_batch_kernel<K>, dim3(blocks), dim3(wg), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_walk_batch(const mcnegf_batch& b, uint64_t seed, uint32_t walker_begin,
                             uint32_t n_walkers, uint32_t max_steps, const mcnegf_walk_config& c,
                             int64_t* tally_override, hipStream_t s) {
    if (n_walkers == 0 || b.n_units == 0) return hipSuccess;
    WalkBatchArgs A;
    A.units = static_cast<const WalkUnit*>(b.d_units);
    A.n_units = b.n_units;
    A.key0 = (uint32_t)(seed & 0xffffffffu);
    A.key1 = (uint32_t)(seed >> 32);
    A.wbegin = walker_begin;
    A.wend = walker_begin + n_walkers;
    A.max_steps = max_steps;
    A.groups = (uint32_t)c.groups;
    A.tally_override = tally_override;
    A.chunk_start = nullptr;
    // chunk: c.chunk walkers, or about `walks_per_slot` walks per slot of a wavefront
    uint64_t ch = c.chunk > 0 ? (uint64_t)c.chunk
                              : (uint64_t)64 * (uint64_t)c.slots * (uint64_t)c.walks_per_slot;
    if (ch > n_walkers) ch = n_walkers;
    A.chunk = (uint32_t)ch;
    A.chunks_per_unit = (uint32_t)((n_walkers + ch - 1) / ch);
    int dev = 0, cus = 0;
    hipError_t err;
    if ((err = hipGetDevice(&dev)) != hipSuccess) return err;
    if ((err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
        hipSuccess)
        return err;
    const void* fn = c.slots == 1   ? (const void*)walk_batch_kernel<1>
                     : c.slots == 2 ? (const void*)walk_batch_kernel<2>
                     : c.slots == 3 ? (const void*)walk_batch_kernel<3>
                                    : (const void*)walk_batch_kernel<4>;
    int per_cu = 0;
    if ((err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, c.wg_size, 0)) !=
        hipSuccess)
        return err;
    // persistent grid: every resident workgroup slot, rounded to whole groups, but no more
    // wavefronts than chunks
    const uint64_t wpb = (uint64_t)c.wg_size / 64;
    uint64_t blocks = (uint64_t)(per_cu < 1 ? 1 : per_cu) * (uint64_t)cus;
    const uint64_t chunks = (uint64_t)A.n_units * A.chunks_per_unit;
    const uint64_t need = (chunks + wpb - 1) / wpb;
    if (blocks > need) blocks = need;
    blocks = (blocks + A.groups - 1) / A.groups * A.groups;
    switch (c.slots) {
        case 1: return launch_walk_batch_k<1>(A, (uint32_t)blocks, (uint32_t)c.wg_size, s);
        case 2: return launch_walk_batch_k<2>(A, (uint32_t)blocks, (uint32_t)c.wg_size, s);
        case 3: return launch_walk_batch_k<3>(A, (uint32_t)blocks, (uint32_t)c.wg_size, s);
        case 4: return launch_walk_batch_k<4>(A, (uint32_t)blocks, (uint32_t)c.wg_size, s);
        default: return hipErrorInvalidValue;
    }
}

// ---- interpolated walks (Sec. V A, "Interpolation") ----------------------------------------
//
// Fine energy f lies between the built energies E_lo <= E_f < E_hi (interp_bracket); its step-6'
// rows are (1 - alpha) p(E_lo) + alpha p(E_hi), a mixture: step n of walker w takes one Philox
// block of counter (n, w, f | 2^31, tag), uses words 0 and 1 as (a, b) of the alias draw and
// draws from E_hi's table when word 2 is below the 32-bit threshold of alpha, else from E_lo's
// (Lemire redraws: counter (n, w, f | 2^31, tag | 2^31), key (key0, key1 ^ r)).  The fine
// energies are the units of a persistent launch: a wavefront walks one chunk of one fine
// energy at a time, with the unit's two tables in scalar registers, and adds the chunk's
// counts to the fine energy's tallies.
struct InterpArgs {
    const uint32_t* tables;  // packed entries of every built energy
    const uint16_t* lows;
    int64_t table_stride;    // entries per energy
    const double* nodes;     // [nE] built energies, ascending
    const double* fine;      // [nF]
    uint32_t nE, nF, pitch, n_out, N;
    uint32_t key0, key1, tag;
    uint32_t wbegin, wend, chunk, chunks_per_unit;
    uint32_t max_steps;
    int64_t* tallies;  // [nF][5]
    uint32_t* status;
};

template <int K>
__global__ void __launch_bounds__(256) walk_interp_kernel(InterpArgs A) {
    const int lane = threadIdx.x & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t wpb = blockDim.x >> 6;
    const uint32_t waves = __builtin_amdgcn_readfirstlane(gridDim.x * wpb);
    const uint32_t lw = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x >> 6));
    const uint32_t total = A.nF * A.chunks_per_unit;
    const uint32_t n_out = A.n_out, N = A.N;
    const uint32_t thresh = (0u - n_out) % n_out;
    const uint32_t inject_row = N + (A.tag & 1u);
    for (uint32_t cid0 = lw; cid0 < total; cid0 += waves) {  // uniform loop
        const uint32_t cid = __builtin_amdgcn_readfirstlane(cid0);
        const uint32_t f = cid / A.chunks_per_unit;
        uint32_t lo, a32;
        bool bad;
        interp_bracket(A.nodes, A.nE, A.fine[f], lo, a32, bad);
        lo = __builtin_amdgcn_readfirstlane(lo);
        a32 = __builtin_amdgcn_readfirstlane(a32);
        const uint32_t hi = lo + 1 < A.nE ? lo + 1 : lo;
        const uint32_t* t_lo = (const uint32_t*)uniform_ptr(A.tables + (size_t)lo * A.table_stride);
        const uint32_t* t_hi = (const uint32_t*)uniform_ptr(A.tables + (size_t)hi * A.table_stride);
        const uint16_t* l_lo = (const uint16_t*)uniform_ptr(A.lows + (size_t)lo * A.table_stride);
        const uint16_t* l_hi = (const uint16_t*)uniform_ptr(A.lows + (size_t)hi * A.table_stride);
        const uint32_t fe = f | 0x80000000u;
        uint32_t next = A.wbegin + (cid - f * A.chunks_per_unit) * A.chunk;
        const uint32_t wend = (uint32_t)min((uint64_t)next + A.chunk, (uint64_t)A.wend);
        Step st[K];
        uint32_t w[K];
        uint32_t cL = 0, cR = 0, tr = 0;
        uint64_t s1 = 0, s2 = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            st[k] = Step{inject_row, 0u, false};
            w[k] = 0u;
        }
        for (;;) {
            // refill idle slots (slot-major, then lane order) from the chunk
            if (next < wend) {
                uint64_t need[K];
#pragma unroll
                for (int k = 0; k < K; ++k) need[k] = __ballot(!st[k].active);
                const uint32_t avail = wend - next;
                uint32_t base = 0;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const uint32_t before = base + __popcll(need[k] & lt_mask);
                    const bool take = !st[k].active && before < avail;
                    count_ended_lane(cL, cR, tr, s1, s2, take && st[k].n != 0u, st[k], N);
                    w[k] = take ? next + before : w[k];
                    st[k].s = take ? inject_row : st[k].s;
                    st[k].n = take ? 0u : st[k].n;
                    st[k].active = st[k].active || take;
                    base += __popcll(need[k]);
                }
                next += base < avail ? base : avail;
            }
            uint64_t any = 0ull;
#pragma unroll
            for (int k = 0; k < K; ++k) any |= __ballot(st[k].active);
            if (any == 0ull) break;
            uint32_t bw[K];
            bool up[K];
            uint64_t m[K];
            bool rej[K];
            uint64_t rb = 0ull;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const Philox4 x = philox4x32_10(st[k].n, w[k], fe, A.tag, A.key0, A.key1);
                bw[k] = x.x[1];
                up[k] = x.x[2] < a32;
                m[k] = (uint64_t)x.x[0] * n_out;
                rej[k] = st[k].active && ((uint32_t)m[k] < thresh);
                rb |= __ballot(rej[k]);
            }
            uint32_t r = 0;
            while (rb != 0ull) {  // rare; uniform loop
                ++r;
                rb = 0ull;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const uint32_t a2 = philox4x32_10(st[k].n, w[k], fe, A.tag | 0x80000000u,
                                                      A.key0, A.key1 ^ r).x[0];
                    const uint64_t m2 = (uint64_t)a2 * n_out;
                    m[k] = rej[k] ? m2 : m[k];
                    rej[k] = rej[k] && ((uint32_t)m2 < thresh);
                    rb |= __ballot(rej[k]);
                }
            }
            uint32_t c[K], at[K], ent[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                c[k] = (uint32_t)(m[k] >> 32);
                at[k] = __umul24(st[k].s, A.pitch) + c[k];
                ent[k] = 0u;
            }
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (st[k].active) ent[k] = (up[k] ? t_hi : t_lo)[at[k]];
            bool keep[K], tie[K];
            uint64_t tb = 0ull;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                keep[k] = (bw[k] >> kAliasIdxBits) < (ent[k] >> kAliasIdxBits);
                tie[k] = st[k].active && (bw[k] >> kAliasIdxBits) == (ent[k] >> kAliasIdxBits);
                tb |= __ballot(tie[k]);
            }
            if (tb != 0ull) {  // rare; uniform branch
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const uint32_t lo16 = tie[k] ? (uint32_t)(up[k] ? l_hi : l_lo)[at[k]] : 0u;
                    keep[k] = tie[k] ? (bw[k] & kAliasIdxMask) < lo16 : keep[k];
                }
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t nxt = keep[k] ? c[k] : (ent[k] & kAliasIdxMask);
                const uint32_t n1 = st[k].n + 1;
                const bool active = st[k].active;
                const bool ends = nxt >= N || n1 >= A.max_steps;
                st[k].s = active ? nxt : st[k].s;
                st[k].n = active ? n1 : st[k].n;
                st[k].active = active && !ends;
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) count_ended_lane(cL, cR, tr, s1, s2, st[k].n != 0u, st[k], N);
        const uint64_t v0 = wave_sum_u64(cL), v1 = wave_sum_u64(cR), v2 = wave_sum_u64(tr);
        const uint64_t v3 = wave_sum_u64(s1), v4 = wave_sum_u64(s2);
        unsigned long long* gt =
            reinterpret_cast<unsigned long long*>(A.tallies + (size_t)f * MCNEGF_TALLY_N);
        if (lane == 0) {
            if (v0) atomicAdd(gt + MCNEGF_TALLY_EXIT_L, (unsigned long long)v0);
            if (v1) atomicAdd(gt + MCNEGF_TALLY_EXIT_R, (unsigned long long)v1);
            if (v2) atomicAdd(gt + MCNEGF_TALLY_TRUNC, (unsigned long long)v2);
            if (v3) atomicAdd(gt + MCNEGF_TALLY_STEPS, (unsigned long long)v3);
            if (v4) atomicAdd(gt + MCNEGF_TALLY_STEPS2, (unsigned long long)v4);
            if (v2) atomicOr(A.status, MCNEGF_FLAG_TRUNC);
            if (bad) atomicOr(A.status, MCNEGF_FLAG_RANGE);
        }
    }
}

hipError_t launch_walk_interp(const mcnegf_kernel& k, const double* fine, uint32_t nF,
                              uint64_t seed, uint32_t tag, uint32_t walker_begin,
                              uint32_t n_walkers, uint32_t max_steps, int64_t* tallies,
                              hipStream_t s) {
    if (n_walkers == 0 || nF == 0) return hipSuccess;
    constexpr int K = 3;
    InterpArgs A;
    A.table_stride = (int64_t)k.n_out * k.alias_pitch;
    A.tables = k.alias;
    A.lows = k.alias_lo;
    A.nodes = k.energies;
    A.fine = fine;
    A.nE = (uint32_t)k.nE;
    A.nF = nF;
    A.pitch = (uint32_t)k.alias_pitch;
    A.n_out = (uint32_t)k.n_out;
    A.N = (uint32_t)k.N;
    A.key0 = (uint32_t)(seed & 0xffffffffu);
    A.key1 = (uint32_t)(seed >> 32);
    A.tag = tag;
    A.wbegin = walker_begin;
    A.wend = walker_begin + n_walkers;
    uint64_t ch = 64ull * K * 8;
    if (ch > n_walkers) ch = n_walkers;
    A.chunk = (uint32_t)ch;
    A.chunks_per_unit = (uint32_t)((n_walkers + ch - 1) / ch);
    A.max_steps = max_steps;
    A.tallies = tallies;
    A.status = k.status;
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t err;
    if ((err = hipGetDevice(&dev)) != hipSuccess) return err;
    if ((err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
        hipSuccess)
        return err;
    if ((err = hipOccupancyMaxActiveBlocksPerMultiprocessor(
             &per_cu, (const void*)walk_interp_kernel<K>, 256, 0)) != hipSuccess)
        return err;
    uint64_t blocks = (uint64_t)(per_cu < 1 ? 1 : per_cu) * (uint64_t)cus;
    const uint64_t chunks = (uint64_t)nF * A.chunks_per_unit;
    const uint64_t need = (chunks + 3) / 4;
    if (blocks > need) blocks = need;
    {
        MCNEGF_TIMED("walk_interp_kernel", s);
        hipLaunchKernelGGL(walk_interp_kernel<K>, dim3((unsigned)blocks), dim3(256), 0, s, A);
    }
    return hipGetLastError();
}

// ---- energies drawn from the weights (importance sampling of E_0, Sec. II F step 2) ------
//
// Walker w (global index) draws its energy from p_k = w_k / sum_j w_j with the Philox block of
// counter (0, w, 0xFFFFFFFF, tag) — an energy index no walk step uses — as the 53-bit uniform u
// of words 0-1: energy = the first k with cdf_{k+1} > u cdf_nE.  The walkers are then sorted by
// energy (counting sort: block histograms, a scan per energy, a scatter) and walked by
// walk_batch_kernel with one unit per energy whose walker indices are its sorted list; a walker
// keeps its global index w in the walk's counters, so the result depends only on the seed,
// tag and walker range.  Everything runs on the device (no host round trip).

// cdf[0] = 0, cdf[k + 1] = cdf[k] + w_k; a negative or non-finite weight counts as 0 and sets
// NONFINITE, as does a zero total.
__global__ void energy_cdf_kernel(const double* __restrict__ w, int nE, double* __restrict__ cdf,
                                  uint32_t* __restrict__ status) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double c = 0.0;
    bool bad = false;
    cdf[0] = 0.0;
    for (int k = 0; k < nE; ++k) {
        double v = w[k];
        if (!(v >= 0.0) || !isfinite(v)) {
            bad = true;
            v = 0.0;
        }
        c += v;
        cdf[k + 1] = c;
    }
    if (bad || !(c > 0.0)) atomicOr(status, MCNEGF_FLAG_NONFINITE);
}

// Block b draws the energies of walkers [b per, (b + 1) per) and writes its histogram
// blockhist[k][b].
__global__ void __launch_bounds__(256) energy_draw_kernel(const double* __restrict__ cdf, int nE,
                                                          uint32_t key0, uint32_t key1,
                                                          uint32_t tag, uint32_t wbegin,
                                                          uint32_t n, uint32_t per, int nblk,
                                                          uint32_t* __restrict__ blockhist,
                                                          uint32_t* __restrict__ draws) {
    extern __shared__ uint32_t hist[];
    const int b = blockIdx.x;
    for (int k = threadIdx.x; k < nE; k += 256) hist[k] = 0u;
    __syncthreads();
    const double total = cdf[nE];
    const uint32_t i0 = (uint32_t)min((uint64_t)b * per, (uint64_t)n);
    const uint32_t i1 = (uint32_t)min((uint64_t)i0 + per, (uint64_t)n);
    for (uint32_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const Philox4 x = philox4x32_10(0u, wbegin + i, 0xFFFFFFFFu, tag, key0, key1);
        const uint64_t bits = (((uint64_t)x.x[0] << 32) | x.x[1]) >> 11;
        const double target = (double)bits * 0x1.0p-53 * total;
        int lo = 0, hi = nE - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cdf[mid + 1] > target) hi = mid; else lo = mid + 1;
        }
        draws[i] = (uint32_t)lo;
        atomicAdd(&hist[lo], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nE; k += 256) blockhist[(size_t)k * nblk + b] = hist[k];
}

// Per energy k (one thread): blockoff[k][b] = sum_{b' < b} blockhist[k][b'], counts[k].
__global__ void energy_scan_kernel(const uint32_t* __restrict__ blockhist, int nE, int nblk,
                                   uint32_t* __restrict__ blockoff, uint32_t* __restrict__ counts) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nE) return;
    uint32_t c = 0;
    for (int b = 0; b < nblk; ++b) {
        blockoff[(size_t)k * nblk + b] = c;
        c += blockhist[(size_t)k * nblk + b];
    }
    counts[k] = c;
}

// One thread: base[k] (first position of energy k in the sorted list), chunk_start[k] and the
// unit descriptors of every energy.
__global__ void energy_units_kernel(const uint32_t* __restrict__ counts, int nE, uint32_t chunk,
                                    uint32_t* __restrict__ base, uint32_t* __restrict__ chunk_start,
                                    WalkUnit* __restrict__ units, const uint32_t* alias,
                                    const uint16_t* alias_lo, int64_t pitch, uint32_t n_out,
                                    uint32_t N, uint32_t tag, int64_t* tallies, uint32_t* status,
                                    const uint32_t* ids) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint32_t pos = 0, ch = 0;
    const size_t stride = (size_t)n_out * (size_t)pitch;
    for (int k = 0; k < nE; ++k) {
        base[k] = pos;
        chunk_start[k] = ch;
        WalkUnit U;
        U.tables = alias + (size_t)k * stride;
        U.lows = alias_lo + (size_t)k * stride;
        U.tally = tallies + (size_t)k * MCNEGF_TALLY_N;
        U.status = status;
        U.ids = ids + pos;
        U.pitch = (uint32_t)pitch;
        U.n_out = n_out;
        U.N = N;
        U.e = (uint32_t)k;
        U.tag = tag;
        U.nw = counts[k];
        units[k] = U;
        pos += counts[k];
        ch += (counts[k] + chunk - 1) / chunk;
    }
    base[nE] = pos;
    chunk_start[nE] = ch;
}

// Block b writes the indices of its walkers into their energies' lists.
__global__ void __launch_bounds__(256) energy_scatter_kernel(const uint32_t* __restrict__ draws,
                                                             int nE, uint32_t wbegin, uint32_t n,
                                                             uint32_t per, int nblk,
                                                             const uint32_t* __restrict__ base,
                                                             const uint32_t* __restrict__ blockoff,
                                                             uint32_t* __restrict__ ids) {
    extern __shared__ uint32_t cur[];
    const int b = blockIdx.x;
    for (int k = threadIdx.x; k < nE; k += 256) cur[k] = base[k] + blockoff[(size_t)k * nblk + b];
    __syncthreads();
    const uint32_t i0 = (uint32_t)min((uint64_t)b * per, (uint64_t)n);
    const uint32_t i1 = (uint32_t)min((uint64_t)i0 + per, (uint64_t)n);
    for (uint32_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const uint32_t k = draws[i];
        ids[atomicAdd(&cur[k], 1u)] = wbegin + i;
    }
}

constexpr int kSampledBlocks = 1024;  // draw / scatter blocks (per-block histograms)
constexpr uint32_t kSampledChunk = 64u * 3u * 8u;

uint64_t sampled_scratch_layout(int nE, uint64_t n, SampledScratch* out, void* base) {
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = off;
        off = (off + bytes + 255) & ~uint64_t(255);
        return at;
    };
    const uint64_t oc = take((uint64_t)(nE + 1) * 8);
    const uint64_t oh = take((uint64_t)nE * kSampledBlocks * 4);
    const uint64_t oo = take((uint64_t)nE * kSampledBlocks * 4);
    const uint64_t on = take((uint64_t)nE * 4);
    const uint64_t ob = take((uint64_t)(nE + 1) * 4);
    const uint64_t os = take((uint64_t)(nE + 1) * 4);
    const uint64_t ou = take((uint64_t)nE * sizeof(WalkUnit));
    const uint64_t od = take(n * 4);
    const uint64_t oi = take(n * 4);
    if (out) {
        char* p = static_cast<char*>(base);
        out->cdf = reinterpret_cast<double*>(p + oc);
        out->blockhist = reinterpret_cast<uint32_t*>(p + oh);
        out->blockoff = reinterpret_cast<uint32_t*>(p + oo);
        out->counts = reinterpret_cast<uint32_t*>(p + on);
        out->base = reinterpret_cast<uint32_t*>(p + ob);
        out->chunk_start = reinterpret_cast<uint32_t*>(p + os);
        out->units = p + ou;
        out->draws = reinterpret_cast<uint32_t*>(p + od);
        out->ids = reinterpret_cast<uint32_t*>(p + oi);
    }
    return off;
}

hipError_t launch_walk_sampled(const mcnegf_kernel& k, const SampledScratch& sc, uint64_t seed,
                               uint32_t tag, uint32_t walker_begin, uint32_t n_walkers,
                               uint32_t max_steps, const double* weights, int64_t* tallies,
                               hipStream_t s);

// Fixed scratch of the allocation-free energy-sampled walk (mc_negf_walk_sampled_noalloc):
// each device that runs it holds one copy until the process ends.  In host code `scratch`
// names a host-side stand-in, not a device address; the device address comes from
// hipGetSymbolAddress, once per device, and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[MCNEGF_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_addr[kMaxDevices] = {};

hipError_t static_scratch_address(void** out) {
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        if ((err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return err;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return hipSuccess;
}

// Per-unit counts: unit u walks the walker indices ids[0 .. nw_u) of its descriptor; the
// chunk prefix (device, [n_units + 1]) was written by the caller.  One XCD group.
hipError_t launch_walk_units(const void* d_units, uint32_t n_units, const uint32_t* d_chunk_start,
                             uint32_t total_chunks, uint32_t chunk, uint64_t seed,
                             uint32_t max_steps, hipStream_t s) {
    if (total_chunks == 0) return hipSuccess;
    constexpr int K = 3;
    WalkBatchArgs A;
    A.units = static_cast<const WalkUnit*>(d_units);
    A.n_units = n_units;
    A.key0 = (uint32_t)(seed & 0xffffffffu);
    A.key1 = (uint32_t)(seed >> 32);
    A.wbegin = 0;
    A.wend = 0;
    A.chunk = chunk;
    A.chunks_per_unit = 0;
    A.groups = 1;
    A.max_steps = max_steps;
    A.tally_override = nullptr;
    A.chunk_start = d_chunk_start;
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t err;
    if ((err = hipGetDevice(&dev)) != hipSuccess) return err;
    if ((err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
        hipSuccess)
        return err;
    if ((err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu,
                                                            (const void*)walk_batch_kernel<K>,
                                                            256, 0)) != hipSuccess)
        return err;
    uint64_t blocks = (uint64_t)(per_cu < 1 ? 1 : per_cu) * (uint64_t)cus;
    const uint64_t need = ((uint64_t)total_chunks + 3) / 4;
    if (blocks > need) blocks = need;
    return launch_walk_batch_k<K>(A, (uint32_t)blocks, 256u, s);
}

hipError_t launch_walk_sampled(const mcnegf_kernel& k, const SampledScratch& sc, uint64_t seed,
                               uint32_t tag, uint32_t walker_begin, uint32_t n_walkers,
                               uint32_t max_steps, const double* weights, int64_t* tallies,
                               hipStream_t s) {
    if (n_walkers == 0) return hipSuccess;
    const int nE = k.nE;
    const uint32_t key0 = (uint32_t)(seed & 0xffffffffu), key1 = (uint32_t)(seed >> 32);
    const uint32_t per = (n_walkers + kSampledBlocks - 1) / kSampledBlocks;
    const size_t lds = (size_t)nE * 4;
    hipError_t err;
    {
        MCNEGF_TIMED("energy_cdf_kernel", s);
        hipLaunchKernelGGL(energy_cdf_kernel, dim3(1), dim3(64), 0, s, weights, nE, sc.cdf,
                           k.status);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    {
        MCNEGF_TIMED("energy_draw_kernel", s);
        hipLaunchKernelGGL(energy_draw_kernel, dim3(kSampledBlocks), dim3(256), lds, s, sc.cdf, nE,
                           key0, key1, tag, walker_begin, n_walkers, per, kSampledBlocks,
                           sc.blockhist, sc.draws);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    {
        MCNEGF_TIMED("energy_scan_kernel", s);
        hipLaunchKernelGGL(energy_scan_kernel, dim3((nE + 255) / 256), dim3(256), 0, s,
                           sc.blockhist, nE, kSampledBlocks, sc.blockoff, sc.counts);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    {
        MCNEGF_TIMED("energy_units_kernel", s);
        hipLaunchKernelGGL(energy_units_kernel, dim3(1), dim3(64), 0, s, sc.counts, nE,
                           kSampledChunk, sc.base, sc.chunk_start,
                           static_cast<WalkUnit*>(sc.units), k.alias, k.alias_lo, k.alias_pitch,
                           (uint32_t)k.n_out, (uint32_t)k.N, tag, tallies, k.status, sc.ids);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    {
        MCNEGF_TIMED("energy_scatter_kernel", s);
        hipLaunchKernelGGL(energy_scatter_kernel, dim3(kSampledBlocks), dim3(256), lds, s,
                           sc.draws, nE, walker_begin, n_walkers, per, kSampledBlocks, sc.base,
                           sc.blockoff, sc.ids);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    // persistent grid; the kernel reads the number of chunks from chunk_start[nE]
    return launch_walk_units(sc.units, (uint32_t)nE, sc.chunk_start, 0xFFFFFFFFu, kSampledChunk,
                             seed, max_steps, s);
}

// ---- importance-sampled walks (Sec. V A, "Improved estimator") ------------------------
//
// The tables sample the modified rows p'_ij = p_ij b_j / rho_i (rho_i = sum_j p_ij b_j) and
// each walker carries the likelihood ratio of its path, the product of p_ij / p'_ij =
// rho_i / b_j over its steps i -> j; a walk that exits at the collecting lead q scores that
// product (the estimator's c_p is applied by the current), any other walk scores 0.  The
// draws are those of mc_negf_walk (same counters), so the paths are the plain walker's paths
// on these tables.
//
// Work layout: energy e belongs to group e % groups (one group per XCD with 8 groups, so an
// energy's tables stay in one L2); every wavefront walks one chunk of kWeightedChunk
// consecutive walkers of one energy, its K slots per lane refilling from the chunk in ballot
// order.  That assignment, and with it every sum below, depends only on the walks, not on
// scheduling: counts go to the tallies as integers; each chunk's two score sums (per lane,
// then a fixed butterfly across the wavefront) go to partial[e][chunk] and are added per
// energy in chunk order by weighted_reduce_kernel.
struct WeightedArgs {
    WalkArgs w;                  // tables of the modified rows; stage_inject = 0
    const double* rho;           // [nE][n_out]
    const double* bias;          // [nE][n_out]
    double* partial;             // [nE][chunks][2]
    uint32_t chunks;             // chunks per energy
    uint32_t blocks_per_energy;  // workgroups of 4 wavefronts per energy
};

constexpr uint32_t kWeightedChunk = 2048;
constexpr int kWeightedSlots = 2;

template <int K>
__device__ inline void weighted_steps(Step (&st)[K], const gtable_ptr (&tb)[K],
                                      const uint32_t (&w)[K], const uint32_t (&el)[K],
                                      const uint32_t (&lq)[K], const uint32_t (&a)[K],
                                      const uint32_t (&b)[K], double (&ratio)[K],
                                      const double* rho, const double* bias, uint32_t q,
                                      const WalkArgs& A) {
    uint32_t from[K];
    bool was[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        from[k] = st[k].s;
        was[k] = st[k].active;
    }
    walk_steps<K>(st, tb, w, el, lq, nullptr, a, b, A);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t to = st[k].s;
        // divergent: loads and arithmetic only
        if (was[k] && (to < A.N || to == q)) ratio[k] *= rho[from[k]] / bias[to];
    }
}

template <int K>
__global__ void __launch_bounds__(256) walk_weighted_kernel(WeightedArgs A) {
    const WalkArgs& W = A.w;
    const uint32_t G = W.groups;
    const uint32_t grp = blockIdx.x % G, j = blockIdx.x / G;
    const uint32_t e = grp + G * (j / A.blocks_per_energy);
    const uint32_t cid = (j % A.blocks_per_energy) * 4 + (threadIdx.x >> 6);
    if (e >= W.nE || cid >= A.chunks) return;  // whole wavefronts; the kernel has no barrier
    const int lane = threadIdx.x & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t N = W.N, n_out = W.n_out;
    const uint32_t inject_row = N + (W.tag & 1u);
    const uint32_t q = N + 1u - (W.tag & 1u);
    const double* rho = A.rho + (size_t)e * n_out;
    const double* bias = A.bias + (size_t)e * n_out;
    uint32_t next = W.wbegin + cid * W.chunk;
    const uint32_t wend = (uint32_t)min((uint64_t)next + W.chunk, (uint64_t)W.wend);

    Step st[K];
    uint32_t w[K], el[K], lq[K];
    gtable_ptr tb[K];
    double ratio[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        st[k] = Step{inject_row, 0u, false};
        w[k] = lq[k] = 0u;
        el[k] = e;
        tb[k] = (gtable_ptr)(W.tables + (size_t)e * W.table_stride);
        ratio[k] = 1.0;
    }
    uint32_t cL = 0, cR = 0, tr = 0;
    uint64_t s1 = 0, s2 = 0;
    double sx = 0.0, sx2 = 0.0;
    // a walk that ended in slot k (done: not counted yet) scores its ratio at an exit at q
    auto finish = [&](bool done, const Step& s, double r) {
        count_ended_lane(cL, cR, tr, s1, s2, done, s, N);
        const double v = (done && s.s == q) ? r : 0.0;
        sx += v;
        sx2 += v * v;
    };
    for (;;) {
        if (next < wend) {  // uniform
            uint64_t need[K];
            uint32_t tot = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                need[k] = __ballot(!st[k].active);
                tot += __popcll(need[k]);
            }
            const uint32_t avail = wend - next;
            uint32_t base = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t before = base + __popcll(need[k] & lt_mask);
                const bool take = !st[k].active && before < avail;
                finish(take && st[k].n != 0u, st[k], ratio[k]);
                w[k] = take ? next + before : w[k];
                st[k].s = take ? inject_row : st[k].s;
                st[k].n = take ? 0u : st[k].n;
                st[k].active = st[k].active || take;
                ratio[k] = take ? 1.0 : ratio[k];
                base += __popcll(need[k]);
            }
            next += tot < avail ? tot : avail;
        }
        uint64_t any = 0ull;
#pragma unroll
        for (int k = 0; k < K; ++k) any |= __ballot(st[k].active);
        if (any == 0ull) break;
        uint32_t a0[K], b0[K], a1[K], b1[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const Philox4 x =
                philox4x32_10(st[k].n >> 1, w[k], W.e_off + e, W.tag, W.key0, W.key1);
            a0[k] = x.x[0];
            b0[k] = x.x[1];
            a1[k] = x.x[2];
            b1[k] = x.x[3];
        }
        weighted_steps<K>(st, tb, w, el, lq, a0, b0, ratio, rho, bias, q, W);
        weighted_steps<K>(st, tb, w, el, lq, a1, b1, ratio, rho, bias, q, W);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) finish(st[k].n != 0u, st[k], ratio[k]);
    // wavefront totals by a fixed butterfly (every lane ends with the same bits)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        sx += __shfl_xor(sx, o, 64);
        sx2 += __shfl_xor(sx2, o, 64);
        cL += __shfl_xor(cL, o, 64);
        cR += __shfl_xor(cR, o, 64);
        tr += __shfl_xor(tr, o, 64);
        s1 += __shfl_xor(s1, o, 64);
        s2 += __shfl_xor(s2, o, 64);
    }
    if (lane == 0) {
        unsigned long long* t =
            reinterpret_cast<unsigned long long*>(W.tallies + (size_t)e * MCNEGF_TALLY_N);
        if (cL) atomicAdd(t + MCNEGF_TALLY_EXIT_L, (unsigned long long)cL);
        if (cR) atomicAdd(t + MCNEGF_TALLY_EXIT_R, (unsigned long long)cR);
        if (tr) atomicAdd(t + MCNEGF_TALLY_TRUNC, (unsigned long long)tr);
        if (s1) atomicAdd(t + MCNEGF_TALLY_STEPS, (unsigned long long)s1);
        if (s2) atomicAdd(t + MCNEGF_TALLY_STEPS2, (unsigned long long)s2);
        double* pp = A.partial + ((size_t)e * A.chunks + cid) * 2;
        pp[0] = sx;
        pp[1] = sx2;
        if (tr) atomicOr(W.status, MCNEGF_FLAG_TRUNC);
    }
}

// wsum[e] += the chunk partials of energy e, in chunk order (lane-strided sums, then a fixed
// butterfly).
__global__ void __launch_bounds__(64) weighted_reduce_kernel(const double* __restrict__ partial,
                                                             uint32_t chunks,
                                                             double* __restrict__ wsum) {
    const uint32_t e = blockIdx.x;
    const int lane = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (uint32_t c = lane; c < chunks; c += 64) {
        a += partial[((size_t)e * chunks + c) * 2];
        b += partial[((size_t)e * chunks + c) * 2 + 1];
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if (lane == 0) {
        wsum[2 * (size_t)e] += a;
        wsum[2 * (size_t)e + 1] += b;
    }
}

uint64_t weighted_scratch_bytes(int nE, uint64_t n_walkers) {
    const uint64_t chunks = (n_walkers + kWeightedChunk - 1) / kWeightedChunk;
    return ((uint64_t)nE * chunks * 16 + 255) & ~uint64_t(255);
}

hipError_t launch_walk_weighted(const mcnegf_kernel& k, const uint32_t* tables,
                                const uint16_t* lows, const double* rho, const double* bias,
                                uint64_t seed, uint32_t tag, uint32_t walker_begin,
                                uint32_t n_walkers, uint32_t max_steps, int64_t* tallies,
                                double* wsum, double* partial, hipStream_t s) {
    if (n_walkers == 0) return hipSuccess;
    WeightedArgs A;
    WalkArgs& W = A.w;
    W.table_stride = (int64_t)k.n_out * k.alias_pitch;
    W.tables = tables;
    W.lows = lows;
    W.pitch32 = (uint32_t)k.alias_pitch;
    W.n_out = (uint32_t)k.n_out;
    W.N = (uint32_t)k.N;
    W.nE = (uint32_t)k.nE;
    W.e_off = 0;
    W.key0 = (uint32_t)(seed & 0xffffffffu);
    W.key1 = (uint32_t)(seed >> 32);
    W.tag = tag;
    W.wbegin = walker_begin;
    W.wend = walker_begin + n_walkers;
    W.chunk = kWeightedChunk;
    W.chunks_per_energy = (n_walkers + kWeightedChunk - 1) / kWeightedChunk;
    W.groups = k.nE >= 8 ? 8u : 1u;
    W.max_steps = max_steps;
    W.stage_inject = 0u;
    W.tallies = tallies;
    W.status = k.status;
    A.rho = rho;
    A.bias = bias;
    A.partial = partial;
    A.chunks = W.chunks_per_energy;
    A.blocks_per_energy = (A.chunks + 3) / 4;
    const uint64_t per_group = ((uint64_t)k.nE + W.groups - 1) / W.groups;
    const uint64_t blocks = per_group * W.groups * A.blocks_per_energy;
    if (blocks >= (1ull << 31)) return hipErrorInvalidValue;
    {
        MCNEGF_TIMED("walk_weighted_kernel", s);
        hipLaunchKernelGGL(walk_weighted_kernel<kWeightedSlots>, dim3((uint32_t)blocks),
                           dim3(256), 0, s, A);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    {
        MCNEGF_TIMED("weighted_reduce_kernel", s);
        hipLaunchKernelGGL(weighted_reduce_kernel, dim3(k.nE), dim3(64), 0, s, partial,
                           A.chunks, wsum);
    }
    return hipGetLastError();
}

// ---- transition counts for the score-function gradient ----------------------------------
//
// Each lane walks one walker exactly as mc_negf_walk does (same counters, Lemire redraws,
// packed entries); a walk that exits at the collecting lead q is walked again from its first
// step (the counter-based draws repeat it exactly) and adds one to counts[e][o][s] for each
// step s -> o.  The counts are integers, so the result does not depend on the order of the
// atomic adds.  Lanes walk divergent loops with no cross-lane operation inside; the tallies
// are reduced across the wavefront after every lane has left its loops.
struct CountArgs {
    const uint32_t* tables;
    const uint16_t* lows;
    uint32_t pitch32;
    int64_t table_stride;
    uint32_t n_out, N, nE;
    uint32_t key0, key1, tag;
    uint32_t wbegin, n_walkers, max_steps;
    uint32_t* counts;  // [nE][n_out][n_out], outcome-major
    int64_t* tallies;
    uint32_t* status;
};

// One step of a single walker from row `row` with Philox words (a, b) of step n_step.
__device__ inline uint32_t draw_step(const CountArgs& A, gtable_ptr tb, const uint16_t* lo,
                                     uint32_t row, uint32_t n_step, uint32_t w, uint32_t e,
                                     uint32_t a, uint32_t b) {
    const uint32_t n_out = A.n_out;
    const uint32_t thresh = (0u - n_out) % n_out;
    uint64_t m = (uint64_t)a * n_out;
    uint32_t r = 0;
    while ((uint32_t)m < thresh) {  // per lane, rare
        ++r;
        m = (uint64_t)philox4x32_10(n_step, w, e, A.tag | 0x80000000u, A.key0, A.key1 ^ r).x[0] *
            n_out;
    }
    const uint32_t c = (uint32_t)(m >> 32);
    const uint32_t off = __umul24(row, A.pitch32) + c;
    const uint32_t ent = tb[off];
    bool keep = b < (ent & ~kAliasIdxMask);
    if (((b ^ ent) >> kAliasIdxBits) == 0u) keep = (b & kAliasIdxMask) < (uint32_t)lo[off];
    return keep ? c : (ent & kAliasIdxMask);
}

// The same draw with the first step's injection row staged in LDS (inj, inj_lo: the row of
// the walker's own energy): lanes at step 0 read the bucket's entry there, the others from
// the global table; both take the same bucket and the same keep rule.
__device__ inline uint32_t draw_step_staged(const CountArgs& A, gtable_ptr tb, const uint16_t* lo,
                                            const uint32_t* inj, const uint16_t* inj_lo,
                                            uint32_t row, uint32_t n_step, uint32_t w, uint32_t e,
                                            uint32_t a, uint32_t b) {
    const uint32_t n_out = A.n_out;
    const uint32_t thresh = (0u - n_out) % n_out;
    uint64_t m = (uint64_t)a * n_out;
    uint32_t r = 0;
    while ((uint32_t)m < thresh) {  // per lane, rare
        ++r;
        m = (uint64_t)philox4x32_10(n_step, w, e, A.tag | 0x80000000u, A.key0, A.key1 ^ r).x[0] *
            n_out;
    }
    const uint32_t c = (uint32_t)(m >> 32);
    const bool staged = n_step == 0u;
    const uint32_t off = __umul24(row, A.pitch32) + c;
    const uint32_t ent = staged ? inj[c] : tb[off];
    bool keep = b < (ent & ~kAliasIdxMask);
    if (((b ^ ent) >> kAliasIdxBits) == 0u)
        keep = (b & kAliasIdxMask) < (uint32_t)(staged ? inj_lo[c] : lo[off]);
    return keep ? c : (ent & kAliasIdxMask);
}

__global__ void __launch_bounds__(256) walk_counts_kernel(CountArgs A) {
    const uint32_t e = blockIdx.y;
    const uint64_t wi = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = wi < A.n_walkers;
    const uint32_t w = A.wbegin + (uint32_t)(valid ? wi : 0);
    const uint32_t N = A.N, n = A.n_out;
    const uint32_t p = A.tag & 1u;
    const uint32_t q = N + 1u - p;
    const gtable_ptr tb = (gtable_ptr)(A.tables + (size_t)e * A.table_stride);
    const uint16_t* lo = A.lows + (size_t)e * A.table_stride;
    uint32_t* cnt = A.counts + (size_t)e * n * n;
    uint32_t steps = 0, fin = N;  // final state of the walk (a probe when truncated)
    for (int pass = 0; pass < 2 && valid; ++pass) {
        uint32_t s = N + p;
        steps = 0;
        Philox4 blk;
        bool ended = false;
        while (steps < A.max_steps) {
            if ((steps & 1u) == 0u) blk = philox4x32_10(steps >> 1, w, e, A.tag, A.key0, A.key1);
            const uint32_t a = blk.x[2 * (steps & 1u)], b = blk.x[2 * (steps & 1u) + 1];
            const uint32_t next = draw_step(A, tb, lo, s, steps, w, e, a, b);
            ++steps;
            if (pass == 1) atomicAdd(cnt + (size_t)next * n + s, 1u);
            s = next;
            if (next >= N) {
                ended = true;
                break;
            }
        }
        fin = s;
        if (pass == 0 && !(ended && s == q)) break;
    }
    uint32_t cL = valid && fin == N ? 1u : 0u;
    uint32_t cR = valid && fin == N + 1 ? 1u : 0u;
    uint32_t tr = valid && fin < N ? 1u : 0u;
    uint64_t s1 = valid ? steps : 0u, s2 = valid ? (uint64_t)steps * steps : 0u;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        cL += __shfl_xor(cL, o, 64);
        cR += __shfl_xor(cR, o, 64);
        tr += __shfl_xor(tr, o, 64);
        s1 += __shfl_xor(s1, o, 64);
        s2 += __shfl_xor(s2, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        unsigned long long* t =
            reinterpret_cast<unsigned long long*>(A.tallies + (size_t)e * MCNEGF_TALLY_N);
        if (cL) atomicAdd(t + MCNEGF_TALLY_EXIT_L, (unsigned long long)cL);
        if (cR) atomicAdd(t + MCNEGF_TALLY_EXIT_R, (unsigned long long)cR);
        if (tr) atomicAdd(t + MCNEGF_TALLY_TRUNC, (unsigned long long)tr);
        if (s1) atomicAdd(t + MCNEGF_TALLY_STEPS, (unsigned long long)s1);
        if (s2) atomicAdd(t + MCNEGF_TALLY_STEPS2, (unsigned long long)s2);
        if (tr) atomicOr(A.status, MCNEGF_FLAG_TRUNC);
    }
}

hipError_t launch_walk_counts(const mcnegf_kernel& k, uint64_t seed, uint32_t tag,
                              uint32_t walker_begin, uint32_t n_walkers, uint32_t max_steps,
                              uint32_t* counts, int64_t* tallies, hipStream_t s) {
    if (n_walkers == 0) return hipSuccess;
    CountArgs A;
    A.tables = k.alias;
    A.lows = k.alias_lo;
    A.pitch32 = (uint32_t)k.alias_pitch;
    A.table_stride = (int64_t)k.n_out * k.alias_pitch;
    A.n_out = (uint32_t)k.n_out;
    A.N = (uint32_t)k.N;
    A.nE = (uint32_t)k.nE;
    A.key0 = (uint32_t)(seed & 0xffffffffu);
    A.key1 = (uint32_t)(seed >> 32);
    A.tag = tag;
    A.wbegin = walker_begin;
    A.n_walkers = n_walkers;
    A.max_steps = max_steps;
    A.counts = counts;
    A.tallies = tallies;
    A.status = k.status;
    {
        MCNEGF_TIMED("walk_counts_kernel", s);
        hipLaunchKernelGGL(walk_counts_kernel, dim3((n_walkers + 255) / 256, k.nE), dim3(256), 0,
                           s, A);
    }
    return hipGetLastError();
}

// ---- inelastic walks (Sec. II F, step 7') -------------------------------------------------
//
// After step 6' draws probe i at energy E_n, step 7' draws the next energy (Eq. (74)): with
// the coupling lambda~_i(E, E_n) = sum_k lambda_k delta(E - E_n - Delta_k) (lines on the grid,
// Delta_k = off[k] grid steps) the walk moves to E_n + Delta_k with probability
// x_k / sum x, x_k = lambda_k A_ii(E_n + Delta_k) (zero off the grid), and continues from
// probe i's row at that energy.  The table holds, per (energy, probe), the running sums of x
// on the 2^32 scale: t_k = floor(2^32 cum_k / total); the first k with r < t_k is drawn for
// a 32-bit word r (k = n_lines - 1 if none is).

struct LineArgs {
    const double* Adiag;  // [nE][N]
    uint64_t* table;      // [nE][N][n_lines]
    uint32_t* status;
    int32_t N, nE, n_lines;
    int32_t off[kMaxLines];
    double lam[kMaxLines];
};

__global__ void __launch_bounds__(256) energy_table_kernel(LineArgs A) {
    // plain products and sums in order: a fused multiply-add would round differently from
    // the threshold definition
#pragma clang fp contract(off)
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)A.nE * A.N) return;
    const int e = (int)(idx / A.N), i = (int)(idx % A.N);
    double cum[kMaxLines];
    double c = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxLines; ++k) {
        if (k < A.n_lines) {
            const int en = e + A.off[k];
            const double x = (en >= 0 && en < A.nE) ? A.lam[k] * A.Adiag[(int64_t)en * A.N + i]
                                                     : 0.0;
            c = c + x;
            cum[k] = c;
        }
    }
    const bool ok = c > 0.0 && c < __builtin_inf();
    uint64_t* t = A.table + idx * A.n_lines;
#pragma unroll
    for (int k = 0; k < kMaxLines; ++k)
        if (k < A.n_lines) t[k] = ok ? (uint64_t)(cum[k] / c * 4294967296.0) : (1ull << 32);
    if (!ok) atomicOr(A.status, MCNEGF_FLAG_NONFINITE);
}

hipError_t launch_energy_table(const mcnegf_kernel& k, int n_lines, const int32_t* off,
                               const double* lam, uint64_t* table, hipStream_t s) {
    LineArgs A;
    A.Adiag = k.Adiag;
    A.table = table;
    A.status = k.status;
    A.N = k.N;
    A.nE = k.nE;
    A.n_lines = n_lines;
    for (int j = 0; j < kMaxLines; ++j) {
        A.off[j] = j < n_lines ? off[j] : 0;
        A.lam[j] = j < n_lines ? lam[j] : 0.0;
    }
    const int64_t n = (int64_t)k.nE * k.N;
    {
        MCNEGF_TIMED("energy_table_kernel", s);
        hipLaunchKernelGGL(energy_table_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           s, A);
    }
    return hipGetLastError();
}

// The walk: a walker keeps the random stream of its injection energy e0 (step-6' words and
// Lemire redraws exactly as the elastic walker at e0); the word r of step n's energy draw is
// word (n & 3) of Philox(counter (n >> 2, w, e0, tag), key (~key0, key1)).  With the single
// line Delta = 0 the walk is the elastic walk, step for step.
struct InelasticArgs {
    CountArgs c;             // tables, stream, walkers, tallies, status (counts unused)
    const uint64_t* table;   // [nE][N][n_lines]
    unsigned long long* hist;  // [2][nE][nE]: exits at lead r of walkers from e0 at energy e
    uint32_t gx;               // workgroups per injection energy
    uint32_t staged;           // 1: the injection row of e0 is staged in LDS
    int32_t n_lines;
    int32_t off[kMaxLines];
};

// Walkers per lane: a workgroup walks 256 * kInelasticPerLane walkers of one injection energy
// and flushes its exit-energy histogram (LDS, 2 nE counters) once.
//
// XCD-aware order: workgroups are dealt to the eight XCDs in turn, so workgroup b runs on XCD
// b % 8.  XCD x takes the injection energies x, x + 8, x + 16, ... one after another (gx
// workgroups each): its L2 then serves mostly one energy's table at a time, and lines that
// move by multiples of 8 grid steps stay within the energies of the same XCD.
constexpr uint32_t kInelasticPerLane = 16;

// NL: the number of lines (a compile-time count, so the thresholds and offsets are plain
// registers).  Index arithmetic in 32 bits where it fits: an energy's table has fewer than
// 2^32 entries, and nE N NL < 2^32 (nE <= 4096, N < 2^16, NL <= 8).
template <int NL>
__global__ void __launch_bounds__(256) walk_inelastic_kernel(InelasticArgs A) {
    extern __shared__ uint32_t hsh[];  // [2][nE]
    const CountArgs& C = A.c;
    const uint32_t nE = C.nE, N = C.N;
    const uint32_t xcd = blockIdx.x & 7u, j = blockIdx.x >> 3;
    const uint32_t e0 = xcd + 8u * (j / A.gx), chunk = j % A.gx;
    if (e0 >= nE) return;  // padding of the last round (whole workgroup)
    const uint32_t p = C.tag & 1u;
    // LDS: exit-energy histogram [2][nE], then the injection row of e0 (packed entries and
    // their low threshold bits, pitch of each)
    uint32_t* inj = hsh + 2 * nE;
    uint16_t* inj_lo = reinterpret_cast<uint16_t*>(inj + C.pitch32);
    for (uint32_t b = threadIdx.x; b < 2 * nE; b += blockDim.x) hsh[b] = 0;
    if (A.staged) {
        const size_t row0 = (size_t)e0 * C.table_stride + (size_t)(N + p) * C.pitch32;
        for (uint32_t b = threadIdx.x; b < C.pitch32; b += blockDim.x) {
            inj[b] = C.tables[row0 + b];
            inj_lo[b] = C.lows[row0 + b];
        }
    }
    __syncthreads();
    const uint32_t ekey0 = ~C.key0;
    const uint64_t stride = (uint64_t)A.gx * blockDim.x;
    uint64_t wi = (uint64_t)chunk * blockDim.x + threadIdx.x;
    uint32_t cL = 0, cR = 0, tr = 0;
    uint64_t s1 = 0, s2 = 0;
    bool bad = false;
    // a lane whose walk ends takes its next walker at the next iteration (per-lane state, no
    // cross-lane operation inside the loop)
    bool live = wi < C.n_walkers;
    uint32_t w = C.wbegin + (uint32_t)(live ? wi : 0);
    uint32_t s = N + p, e = e0, steps = 0;
    // Each iteration takes two steps n, n + 1 (n even) of every live lane: both use words of
    // step-6' block n >> 1 and of energy block n >> 2, so one block of each serves the pair.
    // A walk that ends on the first step leaves its lane idle for the second; the next walker
    // starts at the next iteration (with an even step count).
    while (live) {
        const Philox4 blk = philox4x32_10(steps >> 1, w, e0, C.tag, C.key0, C.key1);
        const Philox4 eblk = philox4x32_10(steps >> 2, w, e0, C.tag, ekey0, C.key1);
        const bool high = (steps & 2u) != 0u;  // words 2, 3 of the energy block
        int outcome = -2;  // -2: walking on; -1: truncated or off the grid; 0/1: lead
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (outcome == -2) {
                const uint32_t a = h ? blk.x[2] : blk.x[0], b = h ? blk.x[3] : blk.x[1];
                const uint64_t base = (uint64_t)e * (uint32_t)C.table_stride;
                const gtable_ptr tb = (gtable_ptr)(C.tables + base);
                const uint16_t* lo = C.lows + base;
                // a walk's first step (always the first half of an iteration) reads the staged
                // injection row
                const uint32_t next =
                    h == 0 && A.staged
                        ? draw_step_staged(C, tb, lo, inj, inj_lo, s, steps, w, e0, a, b)
                        : draw_step(C, tb, lo, s, steps, w, e0, a, b);
                ++steps;
                if (next >= N) {
                    outcome = (int)(next - N);
                } else {
                    const uint32_t r = high ? (h ? eblk.x[3] : eblk.x[2])
                                            : (h ? eblk.x[1] : eblk.x[0]);
                    // the thresholds below the last line, loaded together; the first k with
                    // r < t_k by a select chain from the top
                    const uint64_t* t = A.table + (e * N + next) * (uint32_t)NL;
                    uint64_t tv[NL > 1 ? NL - 1 : 1];
#pragma unroll
                    for (int j = 0; j < NL - 1; ++j) tv[j] = t[j];
                    int d = A.off[NL - 1];
#pragma unroll
                    for (int j = NL - 2; j >= 0; --j) d = (uint64_t)r < tv[j] ? A.off[j] : d;
                    const int en = (int)e + d;
                    if (en < 0 || en >= (int)nE) {
                        bad = true;
                        outcome = -1;
                    } else {
                        e = (uint32_t)en;
                        s = next;
                        if (steps >= C.max_steps) outcome = -1;
                    }
                }
            }
        }
        if (outcome != -2) {
            if (outcome == 0) {
                ++cL;
                atomicAdd(&hsh[e], 1u);
            } else if (outcome == 1) {
                ++cR;
                atomicAdd(&hsh[nE + e], 1u);
            } else {
                ++tr;
            }
            s1 += steps;
            s2 += (uint64_t)steps * steps;
            wi += stride;
            live = wi < C.n_walkers;
            w = C.wbegin + (uint32_t)(live ? wi : 0);
            s = N + p;
            e = e0;
            steps = 0;
        }
    }
    __syncthreads();
    uint32_t nbad = bad ? 1u : 0u;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        cL += __shfl_xor(cL, o, 64);
        cR += __shfl_xor(cR, o, 64);
        tr += __shfl_xor(tr, o, 64);
        s1 += __shfl_xor(s1, o, 64);
        s2 += __shfl_xor(s2, o, 64);
        nbad += __shfl_xor(nbad, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        unsigned long long* t =
            reinterpret_cast<unsigned long long*>(C.tallies + (size_t)e0 * MCNEGF_TALLY_N);
        if (cL) atomicAdd(t + MCNEGF_TALLY_EXIT_L, (unsigned long long)cL);
        if (cR) atomicAdd(t + MCNEGF_TALLY_EXIT_R, (unsigned long long)cR);
        if (tr) atomicAdd(t + MCNEGF_TALLY_TRUNC, (unsigned long long)tr);
        if (s1) atomicAdd(t + MCNEGF_TALLY_STEPS, (unsigned long long)s1);
        if (s2) atomicAdd(t + MCNEGF_TALLY_STEPS2, (unsigned long long)s2);
        if (tr > nbad) atomicOr(C.status, MCNEGF_FLAG_TRUNC);
        if (nbad) atomicOr(C.status, MCNEGF_FLAG_RANGE);
    }
    for (uint32_t b = threadIdx.x; b < 2 * nE; b += blockDim.x) {
        const uint32_t v = hsh[b];
        if (v) {
            const uint32_t r = b >= nE ? 1u : 0u, ex = b - r * nE;
            atomicAdd(A.hist + ((size_t)r * nE + e0) * nE + ex, (unsigned long long)v);
        }
    }
}

hipError_t launch_walk_inelastic(const mcnegf_kernel& k, int n_lines, const int32_t* off,
                                 const uint64_t* table, uint64_t seed, uint32_t tag,
                                 uint32_t walker_begin, uint32_t n_walkers, uint32_t max_steps,
                                 int64_t* tallies, int64_t* hist, hipStream_t s) {
    if (n_walkers == 0) return hipSuccess;
    InelasticArgs A;
    CountArgs& C = A.c;
    C.tables = k.alias;
    C.lows = k.alias_lo;
    C.pitch32 = (uint32_t)k.alias_pitch;
    C.table_stride = (int64_t)k.n_out * k.alias_pitch;
    C.n_out = (uint32_t)k.n_out;
    C.N = (uint32_t)k.N;
    C.nE = (uint32_t)k.nE;
    C.key0 = (uint32_t)(seed & 0xffffffffu);
    C.key1 = (uint32_t)(seed >> 32);
    C.tag = tag;
    C.wbegin = walker_begin;
    C.n_walkers = n_walkers;
    C.max_steps = max_steps;
    C.counts = nullptr;
    C.tallies = tallies;
    C.status = k.status;
    A.table = table;
    A.hist = reinterpret_cast<unsigned long long*>(hist);
    A.n_lines = n_lines;
    for (int j = 0; j < kMaxLines; ++j) A.off[j] = j < n_lines ? off[j] : 0;
    const uint64_t per_block = 256ull * kInelasticPerLane;
    // every lane loops over its walkers with the stride of its energy's workgroups, so any
    // gx >= 1 covers them all; gx is capped to keep the grid within 2^31 - 1 workgroups
    const uint64_t rounds = 8ull * (uint64_t)((k.nE + 7) / 8);
    const uint64_t gx = std::min<uint64_t>((n_walkers + per_block - 1) / per_block,
                                           0x7fffffffull / rounds);
    A.gx = (uint32_t)std::max<uint64_t>(gx, 1);
    const uint64_t blocks = rounds * A.gx;
    {
        MCNEGF_TIMED("walk_inelastic_kernel", s);
        const dim3 grid((unsigned)blocks), block(256);
        // the staged row while the LDS stays within the default 64 KB per workgroup
        const size_t lds_hist = (size_t)8 * k.nE, lds_row = (size_t)6 * k.alias_pitch;
        A.staged = lds_hist + lds_row <= 65536 ? 1u : 0u;
        const size_t lds = lds_hist + (A.staged ? lds_row : 0);
        switch (n_lines) {
            case 1: hipLaunchKernelGGL(walk_inelastic_kernel<1>, grid, block, lds, s, A); break;
            case 2: hipLaunchKernelGGL(walk_inelastic_kernel<2>, grid, block, lds, s, A); break;
            case 3: hipLaunchKernelGGL(walk_inelastic_kernel<3>, grid, block, lds, s, A); break;
            case 4: hipLaunchKernelGGL(walk_inelastic_kernel<4>, grid, block, lds, s, A); break;
            case 5: hipLaunchKernelGGL(walk_inelastic_kernel<5>, grid, block, lds, s, A); break;
            case 6: hipLaunchKernelGGL(walk_inelastic_kernel<6>, grid, block, lds, s, A); break;
            case 7: hipLaunchKernelGGL(walk_inelastic_kernel<7>, grid, block, lds, s, A); break;
            default: hipLaunchKernelGGL(walk_inelastic_kernel<8>, grid, block, lds, s, A); break;
        }
    }
    return hipGetLastError();
}

}  // namespace mcnegf
