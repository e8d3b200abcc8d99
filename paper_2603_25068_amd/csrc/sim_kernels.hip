// HIP kernels of the simulator step and its adjoint, written for gfx950
// (wave64).  One wavefront owns one (scenario, link) segment in the link
// phase and one (scenario, node) in the node phase; four wavefronts per
// workgroup.  Nothing here is a dense contraction, so there is no MFMA: the
// step is bound by memory latency and HBM/L2 traffic.
//
// Floating point: agent positions are float and follow one fixed operation
// order (no contraction: the library is built with -ffp-contract=off), so the
// integer decisions they feed (arrival, vacancy, detector crossings) are
// reproducible; utilities, Gumbel noise, token buckets and departure
// accumulators are double.
#include "sim_internal.h"

#include <math.h>

#include <mutex>

namespace sim {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs; remap the block id
// so that each XCD walks one contiguous range of tiles (its L2 then holds
// neighbouring segments).  Bijective on [0, nblocks).
__device__ __forceinline__ int xcd_tile()
{
    const int nb = gridDim.x, b = blockIdx.x;
    const int x = b & 7, k = b >> 3, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + k;
}

// Same mapping for block b of a role that owns nb consecutive blocks whose
// first block id is a multiple of 8 (so b % 8 is still the XCD).
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int x = b & 7, k = b >> 3, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Scenario of work item `item` when items are numbered scenario-major, n per
// scenario: a scalar branch skips the integer division (tens of instructions
// per lane) in the common single-scenario case.
__device__ __forceinline__ int scenario_of(int item, int n, int S)
{
    if (S == 1) return 0;
    return item / n;
}

__device__ __forceinline__ int readlane_i(int v, int src) { return __builtin_amdgcn_readlane(v, src); }

__device__ __forceinline__ double readlane_d(double v, int src)
{
    union { double d; int i[2]; } u;
    u.d = v;
    u.i[0] = __builtin_amdgcn_readlane(u.i[0], src);
    u.i[1] = __builtin_amdgcn_readlane(u.i[1], src);
    return u.d;
}

__device__ __forceinline__ double wave_sum_d(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// One near-tie record (scenario, step, class, agent, link, decision), links
// in the internal numbering (the host maps them back).  Replays carry no log.
__device__ __forceinline__ void tie_record(const Dev &d, int s, int t, int cls, int ag, int link, int dec)
{
    if (!d.tie_log) return;
    const int k = atomicAdd(d.tie_n, 1);
    if (k >= d.tie_cap) return;
    int32_t *r = d.tie_log + 6 * (int64_t)k;
    r[0] = s; r[1] = t; r[2] = cls; r[3] = ag; r[4] = link; r[5] = dec;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the Weyl key schedule.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 product gives both halves (a single v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// counter (agent, step, purpose + 2*block, 0); purpose 0 = link choice with
// one word per candidate, 1 = merge (word 0)
__device__ __forceinline__ void draw4(uint64_t seed, int agent, int step, int purpose, int block, uint32_t w[4])
{
    w[0] = (uint32_t)agent; w[1] = (uint32_t)step; w[2] = (uint32_t)(purpose + 2 * block); w[3] = 0u;
    philox4x32_10(w, (uint32_t)(seed & 0xffffffffull), (uint32_t)(seed >> 32));
}

// Gumbel(0,1) from the top 24 bits: U = (k + 1/2) 2^-24 lies in (0,1).
__device__ __forceinline__ double gumbel_of(uint32_t w)
{
    const double U = ((double)(w >> 8) + 0.5) * (1.0 / 16777216.0);
    return -log(-log(U));
}


// The same draw in single precision, without branches.  With k = w >> 8,
// U = (k + 1/2) 2^-24.  For U < 1/2 the inner value y = -ln U is at least
// ln 2, and U is exact in float, so the hardware log2 (a few ulp) keeps y
// within ~3e-7 relative.  For U >= 1/2, e = 1 - U = (2^25 - 2k - 1) 2^-25 is
// an odd integer below 2^24 times a power of two, exact in float, and
// y = -ln(1 - e) takes Kahan's log1p correction (Goldberg, "What every
// computer scientist should know about floating-point arithmetic", 1991,
// Theorem 4): with u = fl(1 - e), whose distance 1 - u to one is exact,
// -ln(1 - e) = -ln(u) e / (1 - u) to a few ulp, and y = e when u rounds to
// one.  Both halves share one log of u.  The outer log then adds a few ulp of
// |g| <= 18, so |g - g_double| < 1e-5 (checked exhaustively over all 2^24
// values of k).  A decision compares two scores, each within that bound of
// its double value, and is taken on them only when it wins by kFastMargin
// (five times the largest possible error of the difference); otherwise it is
// recomputed with gumbel_of, so every decision equals the double-precision one.
__device__ __forceinline__ float gumbel_fast(uint32_t w)
{
    constexpr float kLn2 = 0.693147180559945f;
    const uint32_t k = w >> 8;
    const bool lower = k < (1u << 23);
    const float U = ((float)k + 0.5f) * (1.0f / 16777216.0f);
    const float e = (float)((1u << 25) - 2u * k - 1u) * (1.0f / 33554432.0f);   // 1 - U on the upper half
    const float u = lower ? U : 1.0f - e;
    const float lnu = __builtin_amdgcn_logf(u) * kLn2;
    const float r = lower ? 1.0f : e * __builtin_amdgcn_rcpf(1.0f - u);
    const float y = (!lower && u == 1.0f) ? e : -lnu * r;
    return -__builtin_amdgcn_logf(y) * kLn2;
}
constexpr double kFastMargin = 1e-4;
constexpr int kChoiceChunk = 8;    // out-links whose route entries, noise and records are requested together

// ---------------------------------------------------------------------------
// Lane groups: a work item (segment or node) is served by G consecutive
// lanes of a wavefront (G = 8, 16, 32 or 64), 256/G items per workgroup.  All
// cross-lane traffic stays inside the group (width-G shuffles, masked
// ballots); loops that contain shuffles have group-uniform trip counts.
// ---------------------------------------------------------------------------
template <int G>
struct Group {
    int gl, gbase;
    __device__ Group() {
        const int l = threadIdx.x & (kWave - 1);
        gl = l & (G - 1);
        gbase = l & ~(G - 1);
    }
    // bits of the group's lanes (bit i = lane i of the group) where p holds
    __device__ __forceinline__ unsigned long long mask(bool p) const {
        const unsigned long long b = __ballot(p);
        if (G == 64) return b;
        return (b >> gbase) & ((1ull << G) - 1ull);
    }
    __device__ __forceinline__ int count(bool p) const {
        const unsigned long long b = __ballot(p);
        if (G == 64) return __popcll(b);
        return __popcll((b >> gbase) & ((1ull << G) - 1ull));
    }
    template <class T>
    __device__ __forceinline__ T sum(T v) const {
        for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
        return v;
    }
};


// The kernels take the state descriptor by value as their first argument, so
// it sits at offset 0 of the kernel argument segment, and split their blocks
// into roles, one per lane-group size, each an inlined copy of the same code.
// Loads of one field in several roles would be merged into one load at the
// kernel's entry and kept live, in spilled scalar registers, through every
// role.  Each role therefore reads the descriptor through its own copy of the
// argument segment pointer, passed through an empty asm statement the
// optimiser cannot see through, so that a role's loads stay inside the role.
// The pointer comes from the segment itself, never from the address of the
// by-value parameter: that address would escape into the asm and force a
// private copy of the descriptor.  Only for kernels whose first argument is
// the descriptor, unmodified (the node, reverse and straight-through kernels;
// the link kernel's roles need few fields and read the argument directly).
__device__ __forceinline__ const Dev &role_args()
{
    using ArgDev = const __attribute__((address_space(4))) Dev;
    ArgDev *p = (ArgDev *)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return *(const Dev *)p;
}

// Counter increments of one node: releases, and five small counts packed as
// 8-bit fields of one word (each at most 2 per lane, so at most 128 per
// group), summed over the lane group, then one atomic per non-zero counter
// into one of kCtrSlots slots (spread by item) so that concurrent items
// rarely hit the same address.
enum { NF_DEPARTED = 0, NF_EXITED, NF_TRANSFERS, NF_TIES, NF_STUCK, NF_N };
__device__ __forceinline__ uint64_t nf_one(int f) { return 1ull << (8 * f); }

template <int G>
__device__ __forceinline__ void add_node_counters(const Dev &d, const Group<G> &g, int s, int item, int released,
                                                  uint64_t small)
{
    released = g.sum(released);
    small = g.sum(small);
    if (g.gl == 0) {
        unsigned long long *c = (unsigned long long *)&d.ctr[((int64_t)s * kCtrSlots + (item % kCtrSlots)) * CTR_N];
        if (released) atomicAdd(c + CTR_RELEASED, (unsigned long long)released);
        constexpr int ctr_of[NF_N] = {CTR_DEPARTED, CTR_EXITED, CTR_TRANSFERS, CTR_TIES, CTR_STUCK};
#pragma unroll
        for (int f = 0; f < NF_N; ++f) {
            const unsigned long long v = (small >> (8 * f)) & 0xffull;
            if (v) atomicAdd(c + ctr_of[f], v);
        }
    }
}


// ---------------------------------------------------------------------------
// Link phase: per (scenario, link) segment, in place on the ring.
//   Newell car-following with the link cap (Methods eq. newell_model; SI-A),
//   position form x' = min(x + u dt, max(x, x_lead - dn/kappa)), x_hat =
//   min(x', L); leader = rank - lanes; arrival (x_hat >= L - 0.01), vacancy
//   (entry slots = lanes - #(x_hat <= dn/kappa)), token accrual (the previous
//   step's idle cap min(B, 1) is applied here, before the accrual), detector
//   crossings, order check; records the heads (agent, destination) for the
//   node phase.
// Links are split by ring capacity into four contiguous id ranges (at most
// kSmallRing slots, kMidRing, kLongRing, larger), served by G, max(G, 16),
// max(G, 32) and 64 lanes, so that a launch holds about as many waves as the
// chip keeps resident and the longest rings get the most lanes.  Each lane group gets an equal share of the block's LDS.
// A segment is staged into LDS
// (a piece of up to bufcap ranks plus the leader halo) with all loads in
// flight at once, then updated from that snapshot: every input is a time-t
// position, so the update is a pure gather.  Pieces of very long segments
// go back to front, so a piece never reads ranks an earlier piece wrote.
// ---------------------------------------------------------------------------
constexpr int kBigLds = 1024;    // LDS floats per wavefront for big segments (link phase)
constexpr int kLinkUnroll = 4;   // staged ranks per lane and round of the link phase

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ float cf_update(float x, float xl, bool has_leader, float vf, float sp, float Lj)
{
    const float xf = x + vf;
    float xn = xf;
    if (has_leader) {
        const float xc = xl - sp;
        const float cc = (x > xc) ? x : xc;
        xn = (xf <= cc) ? xf : cc;
    }
    return (xn > Lj) ? Lj : xn;
}

template <int G, bool TAPE>
__device__ __forceinline__ void link_segment(const Dev &d, const Group<G> &g, int s, int j, int t, int sample_b,
                                             int tape_k, float *buf, int bufcap)
{
    const int gl = g.gl;
    const int seg = s * d.L + j;
    const LinkCf lc = d.lcf[seg];
    const int cap = lc.cap, ln = lc.lanes;
    // ring counters, this link's entry slots and heads: one record (rhead, rtail, slots, nheads)
    const int4 rc4 = *reinterpret_cast<const int4 *>(&d.ls[seg].rhead);
    const int h0 = rc4.x, n_raw = rc4.y - h0;
    const int n = min(n_raw, cap);   // an overflowing ring (flagged below) is never read past its end
    const int64_t base = (int64_t)s * d.ring_total + lc.ring_base;
    const float vf = lc.vf, sp = lc.sp, Lj = lc.L, thr = lc.thr;
    // detector crossings are needed on sampling steps only: skip their loads and counts otherwise
    const int d0 = lc.det & 0xffffff, nd = sample_b >= 0 ? (lc.det >> 24) : 0;
    const int hm = h0 % cap;
    auto slot_of = [&](int r) { const int q = hm + r; return q >= cap ? q - cap : q; };
    // head records (speculatively, lanes below the lane count)
    int hag = -1, hdst = -1, hdidx = 0;
    if (gl < ln && gl < n) {   // the agent's destination travels with it in the ring
        hag = d.ring_agent[base + slot_of(gl)];
        const int2 ax = d.ring_aux[base + slot_of(gl)];
        hdst = ax.x;
        hdidx = ax.y;
    }
    double Bv = 0.0, accv = 0.0, dBv = 0.0;
    int64_t Ev = 0;
    if (gl == 0) {
        Bv = d.ls[seg].B;
        accv = d.acc[seg];
        if (d.dB) dBv = d.dB[seg];
        if (sample_b >= 0) Ev = d.ls[seg].E;
    }
    int64_t tb = -1;
    if (TAPE) {   // a recording step (tape_k >= 0)
        tb = (int64_t)tape_k * d.S * d.ring_total + base;
        // (head, tail, head slot, departure mask): the node phase sets the mask's bits
        if (gl == 0) d.tape_seg[(int64_t)tape_k * d.S * d.L + seg] = make_int4(h0, h0 + n, hm, 0);
    }
    // a ring keeps `lanes` slots free, so an entry slot never aliases a slot live one step earlier
    if (gl == 0 && n_raw > cap - ln) atomicOr(&d.err[ERR_RING_OVERFLOW], 1);
    float dpos[kMaxDetPerLink];
    int dcnt[kMaxDetPerLink];
#pragma unroll
    for (int k = 0; k < kMaxDetPerLink; ++k) {
        dpos[k] = k < nd ? d.det_pos[d.det_list[d0 + k]] : 0.f;
        dcnt[k] = 0;
    }
    int nh = 0, nocc = 0, viol = 0;
    const int piece = bufcap - kMaxLanes;
    for (int hi = n; hi > 0; hi -= piece) {
        const int lo = max(0, hi - piece);
        const int slo = max(0, lo - ln);
        // stage ranks [slo, hi): kLinkUnroll loads in flight per lane per round; a recording replay
        // also copies the time-t position and agent of ranks [lo, hi) to the tape here, with those loads
        for (int r = slo + gl; r < hi; r += kLinkUnroll * G) {
            float v4[kLinkUnroll];
            int a4[kLinkUnroll];
#pragma unroll
            for (int q = 0; q < kLinkUnroll; ++q) {
                const int rr = r + q * G;
                v4[q] = rr < hi ? d.ring_pos[base + slot_of(rr)] : 0.f;
                a4[q] = (TAPE && rr >= lo && rr < hi) ? d.ring_agent[base + slot_of(rr)] : 0;
            }
#pragma unroll
            for (int q = 0; q < kLinkUnroll; ++q) {
                const int rr = r + q * G;
                if (rr >= hi) continue;
                buf[rr - slo] = v4[q];
                if (TAPE && rr >= lo) {
                    d.tape_pos[tb + slot_of(rr)] = v4[q];
                    d.tape_agent[tb + slot_of(rr)] = a4[q];
                }
            }
        }
        wave_lds_sync();
        for (int r0 = lo; r0 < hi; r0 += G) {
            const int r = r0 + gl;
            const bool v = r < hi;
            float x = 0.f, xl = 0.f, xp = INFINITY;
            if (v) {
                x = buf[r - slo];
                if (r >= ln) xl = buf[r - ln - slo];
                if (r > slo) xp = buf[r - 1 - slo];   // the rank ahead, for the order check
            }
            const float xh = cf_update(x, xl, r >= ln, vf, sp, Lj);
            if (v) d.ring_pos[base + slot_of(r)] = xh;
            nh += g.count(v && xh >= thr);
            nocc += g.count(v && xh <= sp);
#pragma unroll
            for (int k = 0; k < kMaxDetPerLink; ++k)
                if (k < nd) dcnt[k] += g.count(v && xh >= dpos[k]);
            // the step's input order (entrants of the previous step included): position descending
            viol += g.count(v && xp < x);
        }
        wave_lds_sync();
    }
    const int h = min(nh, min(ln, d.maxl));
    if (gl == 0) {
        d.ls[seg].B = (Bv > 1.0 ? 1.0 : Bv) + accv;
        // tangent of the level in the multiplier; the idle cap clears it
        if (d.dB) d.dB[seg] = (Bv > 1.0 ? 0.0 : dBv) + (double)d.capacity[j] * (double)ln * d.dt;
        *reinterpret_cast<int2 *>(&d.ls[seg].slots) = make_int2(max(0, ln - nocc), h);
        if (viol)
            atomicAdd((unsigned long long *)&d.ctr[((int64_t)s * kCtrSlots) * CTR_N + CTR_ORDER_VIOL],
                      (unsigned long long)viol);
        if (sample_b >= 0)
            for (int k = 0; k < nd; ++k)
                d.cum[((int64_t)s * d.D + d.det_list[d0 + k]) * d.nb + sample_b] = (int32_t)(Ev + dcnt[k]);
    }
    if (gl < h) d.head_rec[(int64_t)seg * d.maxl + gl] = make_int4(hag, hdst, hdidx, 0);
}

// Kernel timing (only when d.kstamp is set): every wave stores its start and end, read from the
// real-time counter, into its own pair of the launch's record (plain stores, no contention);
// k_stamp_reduce later folds a record into the first start and the last end, the kernel's
// execution interval without the dispatch gaps around it.
__device__ __forceinline__ unsigned long long stamp_begin(const Dev &d)
{
    return d.kstamp ? wall_clock64() : 0ull;
}
__device__ __forceinline__ void stamp_end(const Dev &d, unsigned long long t0)
{
    if (d.kstamp && (threadIdx.x & 63) == 0) {
        const int64_t w = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
        d.kstamp[2 * w] = t0;
        d.kstamp[2 * w + 1] = wall_clock64();
    }
}

// Ring classes as block roles: class c takes lane groups of ring_lanes(c, G); the first two roles'
// block counts are multiples of 8, so every role keeps the XCD pattern.
__host__ __device__ __forceinline__ constexpr int ring_lanes(int c, int G)
{
    return c == 0 ? G : (c == 1 ? (G > 16 ? G : 16) : (c == 2 ? (G > 32 ? G : 32) : 64));
}
__host__ __device__ __forceinline__ int ring_role_blocks(int items, int lanes, bool last)
{
    const int per = 256 / lanes;
    const int b = (items + per - 1) / per;
    return last ? b : ((b + 7) & ~7);
}
__host__ __device__ __forceinline__ int ring_blocks(const Dev &d, int G)
{
    return ring_role_blocks(d.S * d.lc_n[0], ring_lanes(0, G), false) +
           ring_role_blocks(d.S * d.lc_n[1], ring_lanes(1, G), false) +
           ring_role_blocks(d.S * d.lc_n[2], ring_lanes(2, G), false) +
           ring_role_blocks(d.S * d.lc_n[3], ring_lanes(3, G), true);
}
// block b of the launch -> (class, block within the class, blocks of the class)
__device__ __forceinline__ int ring_role(const Dev &d, int G, int &b, int &nblk)
{
    b = (int)blockIdx.x;
    const int b0 = ring_role_blocks(d.S * d.lc_n[0], ring_lanes(0, G), false);
    if (b < b0) { nblk = b0; return 0; }
    b -= b0;
    const int b1 = ring_role_blocks(d.S * d.lc_n[1], ring_lanes(1, G), false);
    if (b < b1) { nblk = b1; return 1; }
    b -= b1;
    const int b2 = ring_role_blocks(d.S * d.lc_n[2], ring_lanes(2, G), false);
    if (b < b2) { nblk = b2; return 2; }
    b -= b2;
    nblk = (int)gridDim.x - b0 - b1 - b2;
    return 3;
}

template <int GC, bool TAPE>
__device__ __forceinline__ void link_role(const Dev &d, int c, int b, int nblk, int t, int sample_b, int tape_k,
                                          float *lds)
{
    const Group<GC> g;
    constexpr int per = 256 / GC;
    constexpr int sbuf = 4 * kBigLds / per;
    const int n = d.S * d.lc_n[c];
    const int item = xcd_remap(b, nblk) * per + (int)threadIdx.x / GC;
    if (item >= n) return;
    const int s = scenario_of(item, d.lc_n[c], d.S);
    int first = 0;
    for (int k = 0; k < c; ++k) first += d.lc_n[k];
    link_segment<GC, TAPE>(d, g, s, first + (item - s * d.lc_n[c]), t, sample_b, tape_k,
                           lds + ((int)threadIdx.x / GC) * sbuf, sbuf);
}

template <int G, bool TAPE>
__device__ __forceinline__ void link_launch(const Dev &d, int t, int sample_b, int tape_k)
{
    __shared__ float lds[4 * kBigLds];
    int b, nblk;
    const int c = ring_role(d, G, b, nblk);
    if (c == 0) link_role<ring_lanes(0, G), TAPE>(d, 0, b, nblk, t, sample_b, tape_k, lds);
    else if (c == 1) link_role<ring_lanes(1, G), TAPE>(d, 1, b, nblk, t, sample_b, tape_k, lds);
    else if (c == 2) link_role<ring_lanes(2, G), TAPE>(d, 2, b, nblk, t, sample_b, tape_k, lds);
    else link_role<ring_lanes(3, G), TAPE>(d, 3, b, nblk, t, sample_b, tape_k, lds);
}

template <int G, bool TAPE>
__global__ __launch_bounds__(256) void k_link(Dev d, int t, int sample_b, int tape_k)
{
    const unsigned long long t0 = stamp_begin(d);
    link_launch<G, TAPE>(d, t, sample_b, tape_k);
    stamp_end(d, t0);
}

// ---------------------------------------------------------------------------
// Node phase: per (scenario, node), one lane group (G >= candidates).
//   Releases into the node's origin queues; route choice of every candidate
//   (heads of the in-links and origin fronts; SI-B link choice: utility
//   beta/c - theta*(t_ff + shortest time from the link's head), hard choice
//   argmax(V + Gumbel), ties to the lower candidate index; a head whose link
//   ends at its destination leaves the network); merge per out-link (top-k
//   by alpha_from + Gumbel, k = entry slots; SI-B merge choice); FIFO resolve
//   of each in-link's heads against its token bucket; grafted transfer:
//   leavers pop from the in-link ring, entrants push at position 0 onto the
//   out-link ring (SI-B eq. transfer; the graft itself lives in the adjoint).
// Candidate lanes: the heads of in-link q take lanes [off_q, off_q + lanes_q),
// then the node's origins (one per-node table gives each lane its in-link and
// head rank, or its origin and first queue entry).  Out-link lanes k <
// out-degree load the out-link's data and publish it in the group's LDS table;
// candidates publish (key, choice, agent) the same way, so choice, merge ranks
// and entry order are plain LDS reads.  A chooser requests the route entries,
// Philox words and out-link records of 8 out-links before its first score.
// Per-node link lists are padded node-major tables, so every lane finds its
// link in the first load, and the second-level loads of all lane roles go out
// as one straight-line batch.  `item` only spreads the counter atomics.
// ---------------------------------------------------------------------------
// Per-group LDS tables of the node phase: what a lane group's out-link lanes and candidate lanes
// publish for the others, read with plain LDS loads (no cross-lane shuffles inside branchy loops).
struct OutRec { double util; int om, head, slots, tail, base, cap; };   // out-link k of the node
struct alignas(16) CandRec { float kf; int ch, ag, pad; };                 // candidate lane e

template <int G>
__device__ __forceinline__ void node_work(const Dev &d, const Group<G> &g, int s, int v, int item, int t, int tape_k,
                                          OutRec *orc, CandRec *crc, double *ckey)
{
    const int gl = g.gl;
    const int maxl = d.maxl;
    const int cnt = d.node_cnt[v];
    const int64_t rbase_v = d.route_base[v];
    const int deg = cnt & 0xff, dego = (cnt >> 8) & 0xff, norg = (cnt >> 16) & 0xff;
    const int ncin = (cnt >> 24) & 0xff;   // head lanes of the in-links (sum of their lane counts)
    const int nc = ncin + norg;
    const int64_t sL = (int64_t)s * d.L;
    int released = 0;
    uint64_t small = 0;   // packed counts (NF_* fields)

    // first-level loads issued together (padded tables need no offsets)
    const int om_raw = d.out_pad[(int64_t)v * d.max_out + min(gl, d.max_out - 1)];
    // (in-link, q | rank << 8) on head lanes, (origin, first queue entry) on origin lanes
    const int2 cm = d.cand[(int64_t)v * d.max_cand + min(gl, d.max_cand - 1)];
    const int jin_res = d.in_pad[(int64_t)v * d.max_in + min(gl, d.max_in - 1)];
    const int off_res = d.in_loff[(int64_t)v * d.max_in + min(gl, d.max_in - 1)];   // first head lane of in-link gl
    const bool head_lane = gl < ncin, org_lane = !head_lane && gl < nc;
    const int qi = head_lane ? (cm.y & 0xff) : 0, hr_r = head_lane ? (cm.y >> 8) : 0;
    // second-level loads of every role, issued together in straight-line code: a lane without the
    // role reads a valid stand-in entry and its result is selected away.  Loads placed under the
    // role branches would wait for one another (the memory counter is in order, so a branch that
    // waits for its own load also waits for every load issued before it).
    const int om_c = max(om_raw, 0), jin_c = max(jin_res, 0), jh_c = head_lane ? cm.x : 0;
    const int org_c = org_lane ? cm.x : 0;
    const int64_t sjh = sL + jh_c;
    const LinkNd oc = d.lnd[sL + om_c];                                       // out-link constants
    const int4 oq = *reinterpret_cast<const int4 *>(&d.ls[sL + om_c].rhead);   // (rhead, rtail, slots, nheads)
    const LinkSt ist = d.ls[sL + jin_c];                                      // in-link state
    const int hnh = d.ls[sjh].nheads;                                         // the head lane's in-link
    const int4 hrec = d.head_rec[sjh * maxl + hr_r];
    const float hal = d.lnd[sjh].alpha;
    const int htl = d.lnd[sjh].tail;
    int orel = 0, odep = 0, oqe = 0;
    if (d.O > 0) {   // origin lanes: release and departure pointers, end of the queue
        orel = d.rel_ptr[s * d.O + org_c];
        odep = d.dep_ptr[s * d.O + org_c];
        oqe = d.q_off[org_c + 1];
    }
    const bool graft = tape_k >= 0 && d.tape_dstg != nullptr;   // admission-graft tape (recording replay)
    double dBj = 0.0;
    if (graft) dBj = gl < deg ? d.dB[sL + jin_c] : 0.0;
    // ---- out-link lanes ----
    const bool out_lane = gl < dego;
    const int om = out_lane ? om_raw : -1, ohead = out_lane ? oc.head : -1;
    const int oslots = out_lane ? oq.z : 0, otail = out_lane ? oq.y : 0;
    const int obase = out_lane ? oc.ring_base : 0, ocap = out_lane ? oc.cap : 1;
    const double outil = out_lane ? oc.util : 0.0;
    // ---- in-link lanes (resolve): everything this lane updates at the end ----
    const bool in_lane = gl < deg;
    const int64_t sjq = in_lane ? sL + jin_c : -1;
    double Bj = in_lane ? ist.B : 0.0;
    const int nhq = in_lane ? ist.nheads : 0, hq0 = in_lane ? ist.rhead : 0;
    const int64_t Eq0 = in_lane ? ist.E : 0;
    const double Bacc = Bj;   // accrued level before this step's tokens
    // ---- candidate of this lane ----
    const bool hv = head_lane && hr_r < hnh;
    int ag = hv ? hrec.x : -1, dst = hv ? hrec.y : -1, didx = hv ? hrec.z : 0;
    const int from = hv ? jh_c : -1, ftail = hv ? htl : -1;
    const double alpha = hv ? (double)hal : 1.0;
    int origin = -1, dp0 = 0;
    if (org_lane) {
        origin = cm.x;
        const int qb = cm.y, qn = oqe - qb;
        const int so = s * d.O + origin;
        const int rel = orel;
        dp0 = odep;
        // the queue front is the entry at the departure pointer whether or not this step releases
        // it: load it before any release is written
        int fa = -1, fdst = -1, fdidx = 0;
        if (dp0 < qn) { fa = d.q_list[qb + dp0]; fdst = d.q_dest[qb + dp0]; fdidx = d.q_didx[qb + dp0]; }
        int newrel = rel;
        double D = 0.0, rr = 1.0;
        const double t1 = (t + 1) * d.dt;
        if (d.fixed_mode) {
            while (newrel < qn && d.q_rstep[qb + newrel] <= (int64_t)t) ++newrel;
        } else {
            // bins are whole numbers of steps: step t lies in bin t / steps_per_bin, and only its
            // neighbours can touch the step through rounding of the bin edges (bins in increasing
            // order, as a sum over all bins would add them)
            double incr = 0.0;
            const double t0 = t * d.dt;
            const int bc = t / d.rate_bin_steps;
            for (int b = max(bc - 1, 0); b <= bc + 1 && b < d.n_rate_bins; ++b) {
                const double lo = fmax(b * d.rate_bin_s, t0), hi = fmin((b + 1) * d.rate_bin_s, t1);
                if (hi > lo) incr += (double)d.rates[((int64_t)s * d.O + origin) * d.n_rate_bins + b] * (hi - lo);
            }
            D = d.Dacc[so] + incr;
            if (incr != 0.0) d.Dacc[so] = D;
            rr = incr / d.dt;
            while (newrel < qn && (double)(newrel + 1) <= D) ++newrel;
        }
        // mark the released agents, four queue entries loaded per round before their writes
        for (int k0 = rel; k0 < newrel; k0 += 4) {
            int a4[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) a4[q] = (k0 + q < newrel) ? d.q_list[qb + k0 + q] : -1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (a4[q] < 0) continue;
                const int64_t ga = (int64_t)s * d.N + a4[q];
                d.status[ga] = AG_QUEUED;
                if (!d.fixed_mode) d.tstar[ga] = t1 - (D - (double)(k0 + q + 1)) / rr;
                d.rel_t[ga] = t;
            }
        }
        if (newrel != rel) d.rel_ptr[so] = newrel;
        released += newrel - rel;
        if (dp0 < newrel) { ag = fa; dst = fdst; didx = fdidx; }
    }
    const bool ste_rec = tape_k >= 0 && d.tape_ste != nullptr;   // straight-through tape (recording replay)
    const int64_t ste_i = ((int64_t)tape_k * d.S + s) * d.n_cand + (ste_rec ? d.cbase[v] : 0) + gl;
    if (g.count(ag >= 0) == 0) {   // nothing to move at this node this step
        if (ste_rec && gl < nc) d.tape_ste[ste_i] = make_int4(-1, 0, -1, -1);
        add_node_counters<G>(d, g, s, item, released, 0);
        return;
    }
    const uint64_t seed = d.seed[s];

    // ---- route choice (group-uniform loop over out-link blocks of 4) ----
    const bool exiting = ag >= 0 && from >= 0 && dst == v;
    const bool chooser = ag >= 0 && !exiting;
    const double *route = d.route + rbase_v + (int64_t)didx * dego;   // this head's row
    // merge-key words: independent of the choice, drawn first so they overlap its loads
    uint32_t wm[4] = {0u, 0u, 0u, 0u};
    if (ag >= 0) draw4(seed, ag, t, 1, 0, wm);
    if (gl < dego) orc[gl] = OutRec{outil, om, ohead, oslots, otail, obase, ocap};
    wave_lds_sync();
    // fast pass on single-precision noise: for each chunk of out-links, every route entry and
    // Philox word of the chunk is requested before the first score, so one memory round trip
    // serves the chunk
    auto choice_fast = [&](double &best, double &second, int &arg, int &argk) {
        best = -INFINITY;
        second = -INFINITY;
        arg = CH_STUCK;
        argk = 0;
        constexpr int CC = G < kChoiceChunk ? G : kChoiceChunk;
        for (int c0 = 0; c0 < dego; c0 += CC) {
            double rt[CC];
            uint32_t w[CC];
#pragma unroll
            for (int q = 0; q < CC; ++q) rt[q] = (chooser && c0 + q < dego) ? route[c0 + q] : INFINITY;
#pragma unroll
            for (int b = 0; b < CC / 4; ++b) {
                if (chooser && c0 + 4 * b < dego) {
                    draw4(seed, ag, t, 0, (c0 >> 2) + b, w + 4 * b);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) w[4 * b + q] = 0u;
                }
            }
            if (!chooser) continue;
            // the chunk's out-link records, all LDS reads issued before the first score
            double ou[CC];
            int oh[CC], oo[CC];
#pragma unroll
            for (int q = 0; q < CC; ++q) {
                const OutRec &o = orc[min(c0 + q, G - 1)];
                ou[q] = o.util;
                oh[q] = o.head;
                oo[q] = o.om;
            }
#pragma unroll
            for (int q = 0; q < CC; ++q) {
                if (c0 + q >= dego) break;
                const bool ok = !((!d.allow_uturn) & (from >= 0) & (oh[q] == ftail)) & (rt[q] < INFINITY);
                const double sc = ou[q] - d.theta * rt[q] + (double)gumbel_fast(w[q]);
                const bool top = ok & (sc > best), sec = ok & !top & (sc > second);
                second = top ? best : (sec ? sc : second);
                best = top ? sc : best;
                arg = top ? oo[q] : arg;
                argk = top ? c0 + q : argk;
            }
        }
    };
    // one pass per out-link block of 4 (the double-precision redo)
    auto choice_pass = [&](bool on, bool exact, double &best, double &second, int &arg, int &argk) {
        best = -INFINITY;
        second = -INFINITY;
        arg = CH_STUCK;
        argk = 0;
        for (int b0 = 0; b0 < dego; b0 += 4) {
            int hk[4], mk[4];
            double uk[4], rt[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int src = min(b0 + q, G - 1);
                hk[q] = __shfl(ohead, src, G);
                mk[q] = __shfl(om, src, G);
                uk[q] = __shfl(outil, src, G);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) rt[q] = (on && b0 + q < dego) ? route[b0 + q] : INFINITY;
            if (on) {
                uint32_t w[4];
                draw4(seed, ag, t, 0, b0 >> 2, w);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (b0 + q >= dego) continue;
                    if (!d.allow_uturn && from >= 0 && hk[q] == ftail) continue;
                    if (!(rt[q] < INFINITY)) continue;
                    const double V = uk[q] - d.theta * rt[q];
                    const double gq = exact ? gumbel_of(w[q]) : (double)gumbel_fast(w[q]);
                    const double sc = V + gq;
                    if (sc > best) { second = best; best = sc; arg = mk[q]; argk = b0 + q; }
                    else if (sc > second) second = sc;
                }
            }
        }
    };
    double best, second;
    int arg, argk;   // chosen link and its index among the node's out-links (the lane holding its data)
    choice_fast(best, second, arg, argk);
    // lanes whose winner is not clear on the fast noise redo the choice in double precision
    const bool redo = chooser && second > -INFINITY && best - second < kFastMargin;
    if (g.count(redo)) {
        double b2, s2;
        int a2, k2;
        choice_pass(redo, true, b2, s2, a2, k2);
        if (redo) { best = b2; second = s2; arg = a2; argk = k2; }
    }
    int ch = CH_NONE;
    if (chooser) {
        ch = arg;
        if (arg >= 0 && second > -INFINITY && best - second < 1e-12 * (1.0 + fabs(best))) {
            small += nf_one(NF_TIES);
            tie_record(d, s, t, TIE_CHOICE, ag, arg, arg);
        }
    } else if (exiting) {
        ch = CH_EXIT;
    }
    // ---- merge: rank among candidates wanting the same link ----
    // Every candidate lane publishes (key, choice, agent); a chooser counts the candidates of its own
    // out-link that precede it in key order.  Fast pass on single-precision keys alpha_from + g' (g'
    // the fast noise): each lies within 1e-5 + 2^-24 |key| of the double-precision key, so while
    // |key| < 512 a difference of two keys is off by less than 8.2e-5 and its sign is exact wherever
    // it exceeds kFastMargin.  A group with a rival pair inside the margin, or a key of 512 or more,
    // ranks again on double-precision keys (ties broken by agent id, and the near-tie log, live only
    // there).  The candidate lanes 0..nc-1 go in chunks of four, each chunk unrolled and
    // branch-free (predicates combine with non-short-circuit & and |, so no record read is placed
    // under a branch) so that its broadcast LDS reads are in flight together; lanes past nc are
    // masked out of the sums.
    constexpr int kCk = 4;
    const float kf = ag >= 0 ? (float)alpha + gumbel_fast(wm[0]) : 0.f;
    const bool act = ag >= 0 && ch >= 0;
    int rank = 0, close = 0;
    bool knear = false;
    crc[gl] = CandRec{kf, ag >= 0 ? ch : CH_NONE, ag, 0};
    wave_lds_sync();
    {
        int rk = 0, kn = act & !(fabsf(kf) < 512.f);
        for (int e0 = 0; e0 < nc; e0 += kCk)
#pragma unroll
        for (int k = 0; k < kCk; ++k) {
            const int e = e0 + k;
            const CandRec o = crc[e & (G - 1)];
            const bool rival = act & (e < nc) & (e != gl) & (o.ch == ch);
            const float diff = o.kf - kf;
            rk += rival & (diff > 0.f);
            kn |= rival & (fabsf(diff) < (float)kFastMargin);
        }
        rank = rk;
        knear = kn != 0;
    }
    const bool exact = g.count(knear) != 0;   // the group's ranks on double-precision keys
    double key = 0.0;
    if (exact) {
        if (ag >= 0) key = alpha + gumbel_of(wm[0]);
        ckey[gl] = key;
        wave_lds_sync();
        const double tol = 1e-12 * (1.0 + fabs(key));
        int rk = 0, cl = 0;
        for (int e0 = 0; e0 < nc; e0 += kCk)
#pragma unroll
        for (int k = 0; k < kCk; ++k) {
            const int e = e0 + k;
            const CandRec o = crc[e & (G - 1)];
            const double diff = ckey[e & (G - 1)] - key;   // exact in sign: a key is ahead iff diff > 0
            const bool rival = act & (e < nc) & (e != gl) & (o.ch == ch);
            const bool ahead = (diff > 0.0) | ((diff == 0.0) & (o.ag < ag));
            rk += rival & ahead;
            cl |= rival & !ahead & (-diff < tol);
        }
        rank = rk;
        close = cl;
    }
    const int sl = ch >= 0 ? orc[argk].slots : 0;
    const int won = (ch >= 0) && rank < sl;
    if (ch >= 0 && close) {
        small += nf_one(NF_TIES);
        tie_record(d, s, t, TIE_MERGE, ag, ch, 1);
    }

    // ---- resolve: lane q < deg walks in-link q's heads in rank order ----
    int np = 0;
    bool stop = false, consumed = false;
    const int cw = ch * 2 + won;   // choice and merge outcome in one word (one shuffle per head)
#pragma unroll
    for (int r = 0; r < kMaxLanes; ++r) {   // nhq <= maxl <= kMaxLanes
        const int x = __shfl(cw, min(off_res + r, G - 1), G);
        const int c2 = x >> 1, w2 = x & 1;
        if (gl < deg && !stop && r < nhq) {
            if (c2 == CH_EXIT) ++np;
            else if (c2 >= 0 && w2 && Bj >= 1.0) { Bj -= 1.0; ++np; consumed = true; }
            else { stop = true; if (c2 == CH_STUCK) small += nf_one(NF_STUCK); }
        }
    }
    if (gl < deg) {
        if (consumed) d.ls[sjq].B = Bj;   // the idle cap min(B, 1) is applied at the next accrual
        if (np) {
            d.ls[sjq].E = Eq0 + np;
            d.ls[sjq].rhead = hq0 + np;
        }
    }
    const int q_of_lane = qi;
    const int np_q = __shfl(np, q_of_lane, G);
    int passed = 0;
    if (head_lane) passed = (ag >= 0) && hr_r < np_q;
    else passed = (origin >= 0 && ag >= 0 && won);

    // ---- entrants per out-link (lane k < dego counts link k's) and each entrant's place in key order ----
    // each lane republishes its choice as an entrant's (CH_NONE if it does not enter); om is -1 on
    // lanes without an out-link, which no entry matches
    const bool entering = passed && ch >= 0;
    wave_lds_sync();
    crc[gl].ch = entering ? ch : CH_NONE;
    wave_lds_sync();
    // (entrants onto one link are rivals of one another, so the fast keys order them unless the group
    // ranked on double-precision keys)
    int nent = 0, erank = 0;
    if (!exact) {
        for (int e0 = 0; e0 < nc; e0 += kCk)
#pragma unroll
        for (int k = 0; k < kCk; ++k) {
            const int e = e0 + k;
            const CandRec o = crc[e & (G - 1)];
            const bool in = e < nc;
            nent += in & (o.ch == om);
            erank += in & entering & (e != gl) & (o.ch == ch) & (o.kf - kf > 0.f);
        }
    } else {
        for (int e0 = 0; e0 < nc; e0 += kCk)
#pragma unroll
        for (int k = 0; k < kCk; ++k) {
            const int e = e0 + k;
            const CandRec o = crc[e & (G - 1)];
            const bool in = e < nc;
            nent += in & (o.ch == om);
            const double diff = ckey[e & (G - 1)] - key;
            erank += in & entering & (e != gl) & (o.ch == ch) & ((diff > 0.0) | ((diff == 0.0) & (o.ag < ag)));
        }
    }
    if (gl < dego && nent) d.ls[sL + om].rtail = otail + nent;
    int tbase = 0, rbase = 0, rcap = 1;
    if (ch >= 0) {
        const OutRec o = orc[argk];
        tbase = o.tail;
        rbase = o.base;
        rcap = o.cap;
    }
    const int64_t ga = (int64_t)s * d.N + (ag >= 0 ? ag : 0);
    const int64_t slot = (int64_t)s * d.ring_total + rbase + (tbase + erank) % rcap;
    // admission graft: a head leaving on a token carries the token's availability
    // time t_tok = (t+1)dt - (B_pre - 1)/(m q n) into its entry position
    // (psi = -u_to t_tok); B_pre = accrued level minus the tokens taken ahead of it
    float gfac = 0.f;
    if (graft) {
        const double Bq = __shfl(Bacc, q_of_lane, G), dBq = __shfl(dBj, q_of_lane, G);
        const int myr = hr_r, myoff = __shfl(off_res, q_of_lane, G);
        int tok = 0;
        for (int r = 0; r < maxl; ++r) {
            const int c2 = __shfl(ch, min(myoff + r, G - 1), G);
            tok += (r < myr && c2 >= 0);
        }
        if (passed && from >= 0 && ch >= 0) {
            const double mm = (double)d.capm[sL + from];
            const double mqn = mm * (double)d.capacity[from] * (double)d.lanes[from];
            if (mqn > 0.0) {
                const double dtdm = -dBq / mqn + (Bq - (double)tok - 1.0) / (mm * mqn);
                gfac = (float)(-(double)d.u[sL + ch] * dtdm);
            }
        }
    }
    if (ste_rec) {   // this candidate's choice, outcome and the ring slot its adjoint will hold at t+1
        const int hq = __shfl(hq0, q_of_lane, G);   // in-link's head counter before this step
        if (gl < nc) {
            int4 rec = make_int4(-1, 0, -1, -1);
            if (ag >= 0 && ch >= 0) {
                int loc = -1;
                if (passed) loc = (int)(slot - (int64_t)s * d.ring_total);
                else if (from >= 0) loc = d.ring_base[from] + (hq + hr_r) % d.cap[from];
                rec = make_int4(ag, argk | (min(sl, 255) << 8) | (passed << 16), from, loc);
            }
            d.tape_ste[ste_i] = rec;
        }
    }
    if (tape_k >= 0 && passed && from >= 0) {   // where each leaving head went (-1: left the network)
        const int64_t ti = ((int64_t)tape_k * d.S * d.L + sL + from) * maxl + hr_r;
        d.tape_dst[ti] = ch >= 0 ? (int32_t)slot : -1;
        if (graft) d.tape_dstg[ti] = gfac;
    }
    if (passed) {
        if (ch >= 0) {
            d.ring_agent[slot] = ag;
            d.ring_aux[slot] = make_int2(dst, didx);
            d.ring_pos[slot] = 0.f;
            if (origin >= 0) {
                d.status[ga] = AG_ON;
                d.dep_t[ga] = t;
                // a departure: its entry order on the link, for the reverse's departure grafts
                // (erank < entry slots <= lanes <= kMaxLanes)
                if (tape_k >= 0) atomicOr(&d.tape_seg[(int64_t)tape_k * d.S * d.L + sL + ch].w, 1 << erank);
                d.dep_ptr[s * d.O + origin] = dp0 + 1;
                small += nf_one(NF_DEPARTED);
            } else {
                small += nf_one(NF_TRANSFERS);
            }
        } else {
            d.status[ga] = AG_EXITED;
            d.exit_t[ga] = t;
            small += nf_one(NF_EXITED);
        }
    }
    add_node_counters<G>(d, g, s, item, released, small);
}

// Node phase launch: nodes are split on the host into classes by the lane
// group that holds their candidates (8, 16, 32 or 64 lanes, never below the
// schedule's floor; each class a contiguous id range); one launch runs the
// four classes as block roles, each role's block range remapped so that
// neighbouring nodes share an XCD.
template <int G>
__device__ __forceinline__ bool node_role(int c, int b, int nblk, int t, int tape_k, OutRec *orc,
                                          CandRec *crc, double *ckey)
{
    const Dev &d = role_args();
    const Group<G> g;
    const int per = 256 / G;
    const int n = d.S * d.nd_n[c];
    const int item = xcd_remap(b, nblk) * per + (int)threadIdx.x / G;
    if (item >= n) return true;
    const int s = scenario_of(item, d.nd_n[c], d.S);
    const int o = (int)threadIdx.x & ~(G - 1);
    node_work<G>(d, g, s, d.nd_begin[c] + (item - s * d.nd_n[c]), item, t, tape_k, orc + o, crc + o, ckey + o);
    return true;
}

__host__ __device__ __forceinline__ int node_role_blocks(int n, int G, bool last)
{
    const int per = 256 / G;
    const int b = (n + per - 1) / per;
    return last ? b : ((b + 7) & ~7);   // inner roles in multiples of 8 keep the XCD pattern
}

__device__ __forceinline__ void node_launch(const Dev &d, int t, int tape_k)
{
    __shared__ OutRec orc[256];
    __shared__ CandRec crc[256];
    __shared__ double ckey[256];   // double-precision merge keys (groups that rank exactly)
    int b = (int)blockIdx.x;
    const int b8 = node_role_blocks(d.S * d.nd_n[0], 8, false);
    if (b < b8) { node_role<8>(0, b, b8, t, tape_k, orc, crc, ckey); return; }
    b -= b8;
    const int b16 = node_role_blocks(d.S * d.nd_n[1], 16, false);
    if (b < b16) { node_role<16>(1, b, b16, t, tape_k, orc, crc, ckey); return; }
    b -= b16;
    const int b32 = node_role_blocks(d.S * d.nd_n[2], 32, false);
    if (b < b32) { node_role<32>(2, b, b32, t, tape_k, orc, crc, ckey); return; }
    b -= b32;
    node_role<64>(3, b, (int)gridDim.x - b8 - b16 - b32, t, tape_k, orc, crc, ckey);
}

__global__ __launch_bounds__(256) void k_node(Dev d, int t, int tape_k)
{
    const unsigned long long t0 = stamp_begin(d);
    node_launch(d, t, tape_k);
    stamp_end(d, t0);
}

// Tape entry without an update (the state at the end of a replay window).
__global__ __launch_bounds__(256) void k_tape_snapshot(Dev d, int tape_k)
{
    const int lane = lane_id();
    const int seg = xcd_tile() * kWavesPerBlock + (threadIdx.x >> 6);
    if (seg >= d.S * d.L) return;
    const int s = seg / d.L, j = seg - s * d.L;
    const int h0 = d.ls[seg].rhead, n = d.ls[seg].rtail - h0, cap = d.cap[j];
    const int64_t base = (int64_t)s * d.ring_total + d.ring_base[j];
    const int64_t tb = (int64_t)tape_k * d.S * d.ring_total + base;
    if (lane == 0) d.tape_seg[(int64_t)tape_k * d.S * d.L + seg] = make_int4(h0, h0 + n, h0 % cap, 0);
    for (int r = lane; r < n; r += kWave) {
        const int slot = (h0 + r) % cap;
        d.tape_pos[tb + slot] = d.ring_pos[base + slot];
        d.tape_agent[tb + slot] = d.ring_agent[base + slot];
    }
}

// ---------------------------------------------------------------------------
// Reverse of step t (tape entry k holds time t, k+1 time t+1), per segment.
// The adjoint lives in a ring-parallel array: an agent keeps its ring slot
// while it is on a link, so adj_ring[slot] holds dL/dx of that slot's agent.
// Input: adj_ring = dL/dx(t+1) for slots live at t+1 (counts sampled at t+1
// included).  Output: adj_ring = dL/dx(t) for this link's slots live at t,
// plus the counts sampled at t; and the departure grafts of agents that
// entered this link during step t.  Branches are recomputed from the taped
// time-t positions with the forward's exact float operations.
//   cap (SI-A eq. tg): dx_hat/dx' = 1 in both branches;
//   transfer (SI-B eq. transfer, SI-C): the entry position carries x_hat, so
//     a leaving head reads the adjoint at its entry slot (taped forward);
//   exit: total travel time falls by (x_hat - sg x_hat)/u of the last link;
//   free: x' = x + u dt; congested: x' = x_lead - dn/kappa; stopped: x' = x.
// Each agent has at most one follower (rank + lanes), so the leader term is
// a gather.  A piece of ranks [lo, hi) is staged in LDS with its leader and
// follower halos; all reads of a piece finish before its writes, and pieces
// go front to back.  Entry slots written in step t never alias slots live at
// t (a ring keeps `lanes` slots free), so concurrent segments do not race.
// init = 1: adj_ring = dL/dx(T) at the final state (no step).
// ---------------------------------------------------------------------------
constexpr int kRevBigLds = 1280;    // LDS words per wavefront (two arrays), split evenly among its lane groups
constexpr int kRevUnroll = 4;       // staged ranks per lane and round of the reverse

template <int G>
__device__ __forceinline__ void reverse_segment(const Dev &d, const Group<G> &g, int s, int j, int t, int tape_k,
                                                int init, float *buf, int bufcap)
{
    const int gl = g.gl;
    const int seg = s * d.L + j;
    const int64_t SL = (int64_t)d.S * d.L;
    const int64_t ek = tape_k * SL + seg;          // tape entry of time t
    const int64_t ek1 = init ? ek : ek + SL;       // of time t+1 (the final state has none)
    // every per-segment value in one straight-line batch: link records, tape counters at t and
    // t+1, and the entry slots of the heads that left, read speculatively by the lanes below maxl
    // (a head that left has rank < lanes <= maxl <= G, so rank gl's is lane gl's)
    const LinkCf lc = d.lcf[seg];
    const RevCf rc = d.rcf[seg];
    const int4 ts = d.tape_seg[ek];                // (head, tail, head slot = head mod cap, departures)
    const int hk = ts.x, tk = ts.y, hm = ts.z;
    const int depm = init ? 0 : ts.w;              // entry orders of this step's departures
    const int hk1 = d.tape_seg[ek1].x;
    const int ds_l = init ? -1 : d.tape_dst[ek * d.maxl + min(gl, d.maxl - 1)];
    const double gTs = d.gT ? d.gT[s] : 0.0;
    const int cap = lc.cap, ln = lc.lanes;
    const int n = min(tk - hk, cap);
    const int npass = init ? 0 : min(hk1 - hk, ln);
    // lane gl's head: its entry slot if it left during step t (-1: it left the network), else -2
    const int dsx = gl < npass ? ds_l : -2;
    const int64_t base = (int64_t)s * d.ring_total + lc.ring_base;
    const int64_t RTS = (int64_t)d.S * d.ring_total;
    const int64_t tb = (int64_t)tape_k * RTS + base;
    const float vf = lc.vf, sp = lc.sp, Lj = lc.L;
    const float uj = rc.u;
    const double dkap = rc.dkap;
    const float exit_adj = (float)(-gTs * rc.inv_u);
    const int64_t sN = (int64_t)s * d.N;
    auto slot_of = [&](int r) { const int q = hm + r; return q >= cap ? q - cap : q; };
    int sb = -1;
    if (d.gQ && d.cbs > 0 && t > 0 && t % d.cbs == 0 && t / d.cbs <= d.nb) sb = t / d.cbs - 1;
    const int d0 = lc.det & 0xffffff, nd = lc.det >> 24;
    const float sc = 5.0f / Lj;
    const int P = bufcap / 2;
    float *xb = buf, *pb = buf + P;
    const int piece = P - 2 * kMaxLanes;
    double gu = 0.0, gk = 0.0, gm = 0.0;
    for (int lo = 0; lo < n; lo += piece) {
        const int hi = min(n, lo + piece);
        const int slo = max(0, lo - ln), shi = min(n, hi + ln);
        // taped positions of [slo, shi) and the adjoints of the x_hat of [lo, shi): kRevUnroll ranks
        // per lane per round with their direct loads in flight together.  A head that left (rank <
        // npass <= lanes <= G: the first round of the first piece, rank gl) reads its adjoint at the
        // entry slot the tape names, or takes the exit term, in the same batch; a piece holds more
        // than G ranks, so no such head lies in a follower halo
        for (int r = slo + gl; r < shi; r += kRevUnroll * G) {
            float x4[kRevUnroll], a4[kRevUnroll], g0 = 0.f;
            // rank r < G: the first round of the first piece, where rank r is lane gl's head
            const bool left = (r < G) & (dsx >= 0), gone = (r < G) & (dsx == -1);
#pragma unroll
            for (int q = 0; q < kRevUnroll; ++q) {
                const int rr = r + q * G;
                const bool in = rr < shi;
                const int sl = in ? slot_of(rr) : 0;
                const int64_t ai = (q == 0 && left) ? (int64_t)dsx : base + sl;
                x4[q] = in ? d.tape_pos[tb + sl] : 0.f;
                const float a = (in && rr >= lo && !init && (q > 0 || !gone)) ? d.adj_ring[ai] : 0.f;
                a4[q] = (q == 0 && gone) ? exit_adj : a;
            }
            // admission-graft factor of a head that left on a token
            if (d.gm && left) g0 = d.tape_dstg[ek * d.maxl + gl];
#pragma unroll
            for (int q = 0; q < kRevUnroll; ++q) {
                const int rr = r + q * G;
                if (rr < shi) xb[rr - slo] = x4[q];
                if (rr < shi && rr >= lo) pb[rr - slo] = a4[q];
            }
            if (d.gm && left) gm += (double)a4[0] * (double)g0;
        }
        if (init) {   // the final state's cotangents, follower halo [hi, shi) included
            for (int r = lo + gl; r < shi; r += G) pb[r - slo] = d.gx ? d.gx[sN + d.tape_agent[tb + slot_of(r)]] : 0.f;
        }
        wave_lds_sync();
        for (int r0 = lo; r0 < hi; r0 += G) {
            const int r = r0 + gl;
            const bool v = r < hi;
            // every LDS read of the rank is issued unconditionally (a lane without the leader,
            // follower or rank reads its own staged entry instead and selects the value away), so the
            // reads are in flight together rather than one wait per branch; the leader (r - ln >= slo)
            // and the follower (r + ln < n <= shi) always lie in the staged piece when they exist
            const int ir = v ? r - slo : 0;
            const bool hl = v & (r >= ln), hf = v & (r + ln < n);
            const int il = hl ? r - ln - slo : ir, ifl = hf ? r + ln - slo : ir;
            const float x = xb[ir], ap = pb[ir], xl = xb[il], xfol = xb[ifl], apf = pb[ifl];
            float anew;
            if (!init) {
                int br = 0;  // 0 free, 1 congested, 2 stopped
                {
                    const float xf = x + vf, xc = xl - sp;
                    const float cc = (x > xc) ? x : xc;
                    const int b = (xf <= cc) ? 0 : ((x > xc) ? 2 : 1);
                    br = hl ? b : 0;
                }
                float af = 0.f;
                {
                    const float ff = xfol + vf, xc = x - sp;
                    const float cc = (xfol > xc) ? xfol : xc;
                    af = (hf & !(ff <= cc) & !(xfol > xc)) ? apf : 0.f;
                }
                anew = (br != 1 ? ap : 0.f) + af;
                gu += (v & (br == 0)) ? d.dt * (double)ap : 0.0;
                gk += (v & (br == 1)) ? dkap * (double)ap : 0.0;
            } else {
                anew = ap;
            }
            if (sb >= 0) {   // a sampling step (rare): the detector values are read here, not held
#pragma unroll
                for (int k = 0; k < kMaxDetPerLink; ++k) {
                    if (k >= nd) break;
                    const int det = d.det_list[d0 + k];
                    const int64_t qi = ((int64_t)s * d.D + det) * d.nb;
                    const float gC = d.gQ[qi + sb] - (sb + 1 < d.nb ? d.gQ[qi + sb + 1] : 0.f);
                    const float z = sc * (x - d.det_pos[det]);
                    const float sg = 1.0f / (1.0f + expf(-z));
                    anew += gC * sc * sg * (1.0f - sg);
                }
            }
            if (v) d.adj_ring[base + slot_of(r)] = anew;
        }
        wave_lds_sync();
    }
    // departure grafts of the agents that entered this link during step t
    // an entrant of entry order e holds rank n + e at t+1 (the ring's free slots); the departures
    // among them are marked in the taped mask, so the agent and its adjoint are read together
    if (d.depg && gl < kMaxLanes && ((depm >> gl) & 1)) {
        const int sl = slot_of(n + gl);
        const int a = d.tape_agent[(int64_t)(tape_k + 1) * RTS + base + sl];
        d.depg[sN + a] = d.adj_ring[base + sl] * uj;
    }
    gu = g.sum(gu);
    gk = g.sum(gk);
    if (d.gm) gm = g.sum(gm);
    // one non-returning atomic per accumulator: this group is the segment's only writer in the
    // launch, so the sum is the plain accumulator + contribution, without a read held in registers
    // (a 32-bit byte offset, so the tail holds one register, not a 64-bit index: every link has at
    // least four ring slots and scenarios x ring slots stay below 2^31, so seg < 2^29)
    if (gl == 0 && !init) {
        const uint32_t off = (uint32_t)seg * 8u;
        unsafeAtomicAdd((double *)((char *)d.gu + off), gu);
        unsafeAtomicAdd((double *)((char *)d.gk + off), gk);
        if (d.gm) unsafeAtomicAdd((double *)((char *)d.gm + off), gm);
    }
}

template <int GC>
__device__ __forceinline__ void reverse_role(int c, int b, int nblk, int t, int tape_k, int init,
                                             float *lds)
{
    const Dev &d = role_args();
    const Group<GC> g;
    constexpr int per = 256 / GC;
    constexpr int sbuf = 4 * kRevBigLds / per;
    static_assert(sbuf / 2 > 2 * kMaxLanes + GC, "reverse staging piece too small");
    const int n = d.S * d.lc_n[c];
    const int item = xcd_remap(b, nblk) * per + (int)threadIdx.x / GC;
    if (item >= n) return;
    const int s = scenario_of(item, d.lc_n[c], d.S);
    int first = 0;
    for (int k = 0; k < c; ++k) first += d.lc_n[k];
    reverse_segment<GC>(d, g, s, first + (item - s * d.lc_n[c]), t, tape_k, init,
                        lds + ((int)threadIdx.x / GC) * sbuf, sbuf);
}

template <int G>
__device__ __forceinline__ void reverse_launch(const Dev &d, int t, int tape_k, int init)
{
    __shared__ float lds[4 * kRevBigLds];
    int b, nblk;
    const int c = ring_role(d, G, b, nblk);
    if (c == 0) reverse_role<ring_lanes(0, G)>(0, b, nblk, t, tape_k, init, lds);
    else if (c == 1) reverse_role<ring_lanes(1, G)>(1, b, nblk, t, tape_k, init, lds);
    else if (c == 2) reverse_role<ring_lanes(2, G)>(2, b, nblk, t, tape_k, init, lds);
    else reverse_role<ring_lanes(3, G)>(3, b, nblk, t, tape_k, init, lds);
}

// six waves per SIMD (at most 80 VGPRs) keep a whole 1M-agent reverse step resident at once
template <int G>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(G < 64 ? 6 : 1)))
void k_reverse(Dev d, int t, int tape_k, int init)
{
    const unsigned long long t0 = stamp_begin(d);
    reverse_launch<G>(d, t, tape_k, init);
    stamp_end(d, t0);
}

// ---------------------------------------------------------------------------
// Straight-through gradients of step t (SI-B), per node, launched before the
// reverse of step t overwrites the adjoints: adj_ring holds dL/dx(t+1).  The
// hard route choices and merge winners of the forward are held; their relaxed
// weights (value 0, gradient of the softmax) enter the transfer update, so a
// candidate whose weight for its chosen link changes by dw changes the loss by
// G dw with
//   G = M adj(entry slot)            if it moved (entry position M + x - sg x),
//   G = -(M + x_hat) adj(own slot)   if it stayed on its in-link,
//   G = 0                            if an origin front stayed.
// Merge onto one link with k winners: k Plackett-Luce stages, stage s a
// softmax of (alpha_from l + g')/tau over the candidates ranked s and below
// (k = 1 is the single-winner merge of the text), l = 1 the candidate's
// relaxed weight of that link.  dL/d(merge utility) of a candidate is the sum
// over its stages of q (G - sum q G) / tau; alpha takes it directly and the
// route weight l takes alpha times it, which flows through the chosen link's
// softmax weight pi = softmax((V + g)/tau) into V_m = beta_m/c_m - theta r_m
// (r_m the link's free-flow time plus the shortest time to the destination).
// One lane group per (scenario, node) in the node classes of the forward;
// every accumulator has this node as its only writer (beta, cost: its
// out-links; alpha: its in-links; theta: its own entry), so the sums are
// deterministic.
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ void ste_work(const Dev &d, const Group<G> &g, int s, int v, int t, int tape_k,
                                         double *sy, double *sg, double *sd, int *sk, int *sr, int *sa)
{
    const int gl = g.gl;
    const int cnt = d.node_cnt[v];
    const int deg = cnt & 0xff, dego = (cnt >> 8) & 0xff, norg = (cnt >> 16) & 0xff;
    const int nc = ((cnt >> 24) & 0xff) + norg;
    const int64_t sL = (int64_t)s * d.L, sR = (int64_t)s * d.ring_total;
    const int4 rc = gl < nc ? d.tape_ste[((int64_t)tape_k * d.S + s) * d.n_cand + d.cbase[v] + gl]
                            : make_int4(-1, 0, -1, -1);
    if (g.count(rc.x >= 0) < 2) return;   // a lone candidate has weight 1 in every softmax
    const int ag = rc.x, argk = rc.y & 0xff, kst = (rc.y >> 8) & 0xff, moved = (rc.y >> 16) & 1;
    const int from = rc.z, loc = rc.w;
    const bool cand = ag >= 0;
    const double tau = d.tau;
    const uint64_t seed = d.seed[s];
    double Gc = 0.0, y = 0.0, al = 1.0;
    int ftail = -1;
    if (cand) {
        if (from >= 0) { al = (double)d.alpha[sL + from]; ftail = d.tail[from]; }
        uint32_t w[4];
        draw4(seed, ag, t, 1, 0, w);
        y = al + gumbel_of(w[0]);
        if (loc >= 0) {
            const double A = (double)d.adj_ring[sR + loc];
            if (moved) {
                Gc = d.big_m * A;
            } else {
                const double xh = (double)d.tape_pos[(int64_t)(tape_k + 1) * d.S * d.ring_total + sR + loc];
                Gc = -(d.big_m + xh) * A;
            }
        }
    }
    sy[gl] = y;
    sg[gl] = Gc;
    sk[gl] = cand ? argk : -1;
    sa[gl] = ag;
    wave_lds_sync();
    // place in the merge order of its target (key descending, agent id on ties) and group size
    int rho = 0, n = 1;
    if (cand) {
        for (int e = 0; e < nc; ++e) {
            if (e == gl || sk[e] != argk) continue;
            ++n;
            const double y2 = sy[e];
            if (y2 > y || (y2 == y && sa[e] < ag)) ++rho;
        }
    }
    sr[gl] = rho;
    wave_lds_sync();
    double dVp = 0.0;
    if (cand && n >= 2) {
        const int K = min(n, kst);
        for (int st = 0; st < K && st <= rho; ++st) {
            double mx = -INFINITY;
            for (int e = 0; e < nc; ++e)
                if (sk[e] == argk && sr[e] >= st) mx = fmax(mx, sy[e] / tau);
            double Z = 0.0, ZG = 0.0;
            for (int e = 0; e < nc; ++e) {
                if (sk[e] != argk || sr[e] < st) continue;
                const double q = exp(sy[e] / tau - mx);
                Z += q;
                ZG += q * sg[e];
            }
            const double q = exp(y / tau - mx) / Z;
            dVp += q / tau * (Gc - ZG / Z);
        }
    }
    sd[gl] = dVp;
    wave_lds_sync();
    if (gl < deg) {   // alpha of in-link gl: its candidate lanes in order
        const int jin = d.in_pad[(int64_t)v * d.max_in + gl];
        const int off = d.in_loff[(int64_t)v * d.max_in + gl], ln = d.lanes[jin];
        double a = 0.0;
        bool any = false;
        for (int r = 0; r < ln; ++r) { a += sd[off + r]; any |= sk[off + r] >= 0; }
        if (any) d.galpha[sL + jin] += a;
    }
    const double gam = al * dVp;
    if (g.count(gam != 0.0) == 0) return;
    // route choice: softmax of (V + g)/tau over the admissible out-links, then dV_m per out-link
    int om = -1, ohead = -1;
    double outil = 0.0;
    if (gl < dego) {
        om = d.out_pad[(int64_t)v * d.max_out + gl];
        ohead = d.head[om];
        outil = d.util[sL + om];
    }
    const double *route = d.route + d.route_base[v] + (int64_t)(cand ? d.agent_didx[ag] : 0) * dego;
    const bool on = cand && gam != 0.0;
    auto scores = [&](int b0, double (&yk)[4], double (&rk)[4]) {
        int hk[4];
        double uk[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int src = min(b0 + q, G - 1);
            hk[q] = __shfl(ohead, src, G);
            uk[q] = __shfl(outil, src, G);
        }
        uint32_t w[4] = {0u, 0u, 0u, 0u};
        if (on) draw4(seed, ag, t, 0, b0 >> 2, w);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            yk[q] = -INFINITY;
            rk[q] = (on && b0 + q < dego) ? route[b0 + q] : INFINITY;
            if (!on || b0 + q >= dego) continue;
            if (!d.allow_uturn && from >= 0 && hk[q] == ftail) continue;
            if (!(rk[q] < INFINITY)) continue;
            yk[q] = (uk[q] - d.theta * rk[q] + gumbel_of(w[q])) / tau;
        }
    };
    double mx = -INFINITY, Z = 0.0, ych = -INFINITY;
    for (int b0 = 0; b0 < dego; b0 += 4) {
        double yk[4], rk[4];
        scores(b0, yk, rk);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (yk[q] == -INFINITY) continue;
            if (b0 + q == argk) ych = yk[q];
            if (yk[q] > mx) { Z = Z * exp(mx - yk[q]) + 1.0; mx = yk[q]; }
            else Z += exp(yk[q] - mx);
        }
    }
    const double ps = on ? exp(ych - mx) / Z : 0.0;   // weight of the chosen link
    double mys = 0.0, th = 0.0;
    for (int b0 = 0; b0 < dego; b0 += 4) {
        double yk[4], rk[4];
        scores(b0, yk, rk);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double dv = 0.0;
            if (yk[q] != -INFINITY) {
                const double p = exp(yk[q] - mx) / Z;
                dv = gam / tau * ps * ((b0 + q == argk ? 1.0 : 0.0) - p);
                th -= rk[q] * dv;
            }
            const double sum = g.sum(dv);
            if (gl == b0 + q) mys = sum;
        }
    }
    if (gl < dego && mys != 0.0) {
        const double c = (double)d.cost[sL + om], b = (double)d.beta[sL + om];
        d.gbeta[sL + om] += mys / c;
        d.gcost[sL + om] -= b / (c * c) * mys;
    }
    th = g.sum(th);
    if (gl == 0) d.gth[(int64_t)s * d.Nn + v] += th;
}

template <int G>
__device__ __forceinline__ void ste_role(int c, int b, int nblk, int t, int tape_k, double *sy,
                                         double *sg, double *sd, int *sk, int *sr, int *sa)
{
    const Dev &d = role_args();
    const Group<G> g;
    const int per = 256 / G;
    const int n = d.S * d.nd_n[c];
    const int item = xcd_remap(b, nblk) * per + (int)threadIdx.x / G;
    if (item >= n) return;
    const int s = scenario_of(item, d.nd_n[c], d.S);
    const int o = (int)threadIdx.x & ~(G - 1);
    ste_work<G>(d, g, s, d.nd_begin[c] + (item - s * d.nd_n[c]), t, tape_k, sy + o, sg + o, sd + o, sk + o, sr + o,
                sa + o);
}

__global__ __launch_bounds__(256) void k_ste(Dev d, int t, int tape_k)
{
    __shared__ double sy[256], sg[256], sd[256];
    __shared__ int sk[256], sr[256], sa[256];
    int b = (int)blockIdx.x;
    const int b8 = node_role_blocks(d.S * d.nd_n[0], 8, false);
    if (b < b8) { ste_role<8>(0, b, b8, t, tape_k, sy, sg, sd, sk, sr, sa); return; }
    b -= b8;
    const int b16 = node_role_blocks(d.S * d.nd_n[1], 16, false);
    if (b < b16) { ste_role<16>(1, b, b16, t, tape_k, sy, sg, sd, sk, sr, sa); return; }
    b -= b16;
    const int b32 = node_role_blocks(d.S * d.nd_n[2], 32, false);
    if (b < b32) { ste_role<32>(2, b, b32, t, tape_k, sy, sg, sd, sk, sr, sa); return; }
    b -= b32;
    ste_role<64>(3, b, (int)gridDim.x - b8 - b16 - b32, t, tape_k, sy, sg, sd, sk, sr, sa);
}

// theta gradient of each scenario: the per-node parts summed in node order by one wavefront
__global__ __launch_bounds__(64) void k_theta_sum(Dev d, float *out)
{
    const int s = blockIdx.x;
    double a = 0.0;
    for (int v = lane_id(); v < d.Nn; v += kWave) a += d.gth[(int64_t)s * d.Nn + v];
    a = wave_sum_d(a);
    if (lane_id() == 0) out[s] = (float)a;
}

// dL/d rates[s, o, b] = sum over departed agents of origin o of
// depg * overlap(bin b, [0, t*)) / rate(release bin): the departure-time
// graft (the entry position moves by u * (change of release time)).
// One wavefront per (scenario, origin), lane = bin, agents in queue order.
__global__ __launch_bounds__(256) void k_rate_grad(Dev d, float *g)
{
    const int lane = lane_id();
    const int wid = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (wid >= d.S * d.O) return;
    const int s = wid / d.O, o = wid - s * d.O;
    const int nbins = d.n_rate_bins;
    const int qb = d.q_off[o], qn = d.q_off[o + 1] - qb;
    const int64_t sN = (int64_t)s * d.N;
    const float *rates = d.rates + ((int64_t)s * d.O + o) * nbins;
    // lanes take the queue's agents 64 at a time; per bin, a fixed-order wave sum (deterministic)
    double accb = 0.0;   // lane b < nbins (in its round of 64 bins) holds bin b's total
    for (int b0 = 0; b0 < nbins; b0 += kWave) {
        accb = 0.0;
        for (int k0 = 0; k0 < qn; k0 += kWave) {
            const int k = k0 + lane;
            double dg = 0.0, rt = 1.0, ts = 0.0;
            if (k < qn) {
                const int a = d.q_list[qb + k];
                if (d.dep_t[sN + a] >= 0) {
                    ts = d.tstar[sN + a];
                    const int rb = min(nbins - 1, max(0, (int)floor((double)d.rel_t[sN + a] * d.dt / d.rate_bin_s)));
                    dg = (double)d.depg[sN + a];
                    rt = (double)rates[rb];
                }
            }
            for (int bb = 0; bb < kWave && b0 + bb < nbins; ++bb) {
                const int b = b0 + bb;
                const double ov = fmin((b + 1) * d.rate_bin_s, ts) - b * d.rate_bin_s;
                double c = (dg != 0.0 && ov > 0) ? dg * ov / rt : 0.0;
                for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
                if (lane == bb) accb += c;
            }
        }
        if (b0 + lane < nbins) g[((int64_t)s * d.O + o) * nbins + b0 + lane] = (float)accb;
    }
}

// Derived per-(scenario, link) constants.
__global__ void k_derive(Dev d, const float *cap_mult, const float *capacity, const float *beta,
                         const float *cost, double *util, double *acc, float *vfree, float *spacing, LinkNd *lnd,
                         LinkCf *lcf, RevCf *rcf)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)d.S * d.L) return;
    const int j = (int)(i % d.L);
    vfree[i] = __fmul_rn(d.u[i], (float)d.dt);
    spacing[i] = __fdiv_rn((float)d.platoon, d.kappa[i]);
    util[i] = (double)beta[i] / (double)cost[i];
    acc[i] = (double)cap_mult[i] * (double)capacity[j] * (double)d.lanes[j] * d.dt;
    LinkNd c;
    c.util = (double)beta[i] / (double)cost[i];
    c.alpha = d.alpha[i];
    c.head = d.head[j];
    c.tail = d.tail[j];
    c.ring_base = d.ring_base[j];
    c.cap = d.cap[j];
    c.lanes = d.lanes[j];
    lnd[i] = c;
    LinkCf f;
    f.vf = vfree[i];
    f.sp = spacing[i];
    f.L = d.length[j];
    f.thr = d.thr[j];
    f.cap = d.cap[j];
    f.lanes = d.lanes[j];
    f.ring_base = d.ring_base[j];
    f.det = d.det_off[j] | ((d.det_off[j + 1] - d.det_off[j]) << 24);
    lcf[i] = f;
    RevCf rv;
    const double kd = (double)d.kappa[i];
    rv.dkap = (double)d.platoon / (kd * kd);
    rv.inv_u = 1.0 / (double)d.u[i];
    rv.u = d.u[i];
    rv.pad = 0;
    rcf[i] = rv;
}

// Total travel time and vehicle-steps per scenario: dt * sum over released
// agents of ((exit step or T) - release step), i.e. agent-steps spent queued
// or on the network after each step, and sum over departed agents of
// ((exit step or T) - departure step), the agent-steps on the network.  One
// workgroup per scenario, fixed reduction order.
// Total travel time and vehicle-steps: integer sums over agents of (exit or T) - release and
// (exit or T) - departure, exact in int64 whatever the order; each block adds its sum with one
// atomic, and k_ttt_final scales by dt.
// The checkpoint's arrays in one launch: 16-byte chunks grid-strided over each array, then its
// byte tail (all arrays start on 256-byte boundaries).
__global__ __launch_bounds__(256) void k_copy_multi(CopyJobs jobs)
{
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nth = (uint64_t)gridDim.x * blockDim.x;
    for (int k = 0; k < jobs.n; ++k) {
        const uint4 *src = static_cast<const uint4 *>(jobs.job[k].src);
        uint4 *dst = static_cast<uint4 *>(jobs.job[k].dst);
        const uint64_t nv = jobs.job[k].bytes / 16, rem = jobs.job[k].bytes - nv * 16;
        for (uint64_t i = tid; i < nv; i += nth) dst[i] = src[i];
        if (tid < rem)
            static_cast<char *>(jobs.job[k].dst)[nv * 16 + tid] =
                static_cast<const char *>(jobs.job[k].src)[nv * 16 + tid];
    }
}

__global__ __launch_bounds__(256) void k_ttt(Dev d, int T, unsigned long long *acc)
{
    const int s = blockIdx.y;
    const int64_t sN = (int64_t)s * d.N;
    long long tt = 0, vs = 0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < d.N; i += gridDim.x * 256) {
        const uint8_t st = d.status[sN + i];
        if (st == AG_WAIT) continue;
        const int e = (st == AG_EXITED) ? d.exit_t[sN + i] : T;
        tt += e - d.rel_t[sN + i];
        if (st != AG_QUEUED) vs += e - (d.dep_t[sN + i] >= 0 ? d.dep_t[sN + i] : 0);  // placed agents: from t = 0
    }
    for (int o = 32; o > 0; o >>= 1) { tt += __shfl_xor(tt, o); vs += __shfl_xor(vs, o); }
    __shared__ long long p[2][kWavesPerBlock];
    if ((threadIdx.x & 63) == 0) { p[0][threadIdx.x >> 6] = tt; p[1][threadIdx.x >> 6] = vs; }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long a = 0, b = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) { a += p[0][w]; b += p[1][w]; }
        atomicAdd(&acc[2 * s], (unsigned long long)a);
        atomicAdd(&acc[2 * s + 1], (unsigned long long)b);
    }
}
__global__ void k_zero_u64(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}
__global__ void k_ttt_final(int S, double dt, const unsigned long long *acc, double *out, int64_t *vsteps)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    out[s] = (double)(long long)acc[2 * s] * dt;
    if (vsteps) vsteps[s] = (int64_t)(long long)acc[2 * s + 1];
}

// Interval counts from cumulative samples.
__global__ void k_counts(Dev d, float *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)d.S * d.D * d.nb) return;
    const int b = (int)(i % d.nb);
    out[i] = (float)(d.cum[i] - (b > 0 ? d.cum[i - 1] : 0));
}

// dst[s, caller link] = src[s, internal link], double -> float
__global__ void k_gather_links(const double *src, const int32_t *linv, float *dst, int S, int L)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)S * L) return;
    const int64_t s = i / L, jo = i - s * L;
    dst[i] = (float)src[s * L + linv[jo]];
}

__global__ void k_d2f(const double *src, float *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

__global__ void k_philox(int n, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
    philox4x32_10(c, key[2 * i], key[2 * i + 1]);
    for (int k = 0; k < 4; ++k) out[4 * i + k] = c[k];
}


// ---------------------------------------------------------------------------
// Segmented sort: keys (segment, position, sequence) -> permutation in
// segment order, position descending, sequence ascending, input index
// ascending.  A counting pass by segment (histogram, scan, scatter) places
// every key in its segment; then one workgroup per segment runs a stable
// LSD radix sort in LDS over the 96-bit key (flipped position bits,
// sequence, index) with 4-bit digits.  Segments up to kSortMax keys.
// ---------------------------------------------------------------------------
constexpr int kSortMax = 2048;
constexpr int kSortThreads = 256;
constexpr int kSortPer = kSortMax / kSortThreads;   // keys per thread

__global__ void k_seg_hist(int n, const int32_t *seg, int32_t *cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&cnt[seg[i]], 1);
}

// single-workgroup exclusive scan of n_seg counts -> off[0..n_seg]
__global__ __launch_bounds__(1024) void k_seg_scan(int n_seg, const int32_t *cnt, int32_t *off, int32_t *cursor)
{
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x;
    const int per = (n_seg + 1023) / 1024;
    const int b = tid * per, e = min(n_seg, b + per);
    int32_t sum = 0;
    for (int i = b; i < e; ++i) sum += cnt[i];
    part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int32_t v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t run = part[tid] - sum;
    for (int i = b; i < e; ++i) { off[i] = run; cursor[i] = run; run += cnt[i]; }
    if (tid == 1023) off[n_seg] = part[1023];
}

__global__ void k_seg_scatter(int n, const int32_t *seg, int32_t *cursor, int32_t *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[atomicAdd(&cursor[seg[i]], 1)] = i;
}

__device__ __forceinline__ uint32_t desc_float_key(float x)
{
    uint32_t u = __float_as_uint(x == 0.0f ? 0.0f : x);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);  // ascending order of x
    return ~u;                                        // descending
}

__global__ __launch_bounds__(kSortThreads) void k_seg_lds_sort(const int32_t *off, const float *pos, const int32_t *seq,
                                                               int32_t *perm, int32_t *err)
{
    __shared__ uint32_t k0[kSortMax], k1[kSortMax], k2[kSortMax];
    __shared__ uint32_t t0[kSortMax], t1[kSortMax], t2[kSortMax];
    __shared__ int32_t cnt[16 * kSortThreads];
    __shared__ int32_t wsum[kSortThreads];
    const int sgi = blockIdx.x, tid = threadIdx.x;
    const int b = off[sgi], n = off[sgi + 1] - b;
    if (n <= 1) return;
    if (n > kSortMax) { if (tid == 0) atomicOr(err, 1); return; }
    for (int i = tid; i < n; i += kSortThreads) {
        const int idx = perm[b + i];
        k0[i] = (uint32_t)idx;                 // least significant
        k1[i] = (uint32_t)seq[idx] ^ 0x80000000u;
        k2[i] = desc_float_key(pos[idx]);      // most significant
    }
    __syncthreads();
    const int lo = tid * kSortPer, hi = min(n, lo + kSortPer);
    for (int pass = 0; pass < 24; ++pass) {
        const int word = pass >> 3, shift = (pass & 7) * 4;
        uint32_t *src = word == 0 ? k0 : (word == 1 ? k1 : k2);
        // per-thread digit counts (digit-major layout keeps the scatter stable)
        for (int dgt = 0; dgt < 16; ++dgt) cnt[dgt * kSortThreads + tid] = 0;
        for (int i = lo; i < hi; ++i) cnt[((src[i] >> shift) & 15u) * kSortThreads + tid] += 1;
        __syncthreads();
        // exclusive scan over the 16*256 counters: thread tid owns counters [16 tid, 16 tid + 16)
        int32_t run = 0;
        for (int q = 0; q < 16; ++q) run += cnt[tid * 16 + q];
        wsum[tid] = run;
        __syncthreads();
        for (int o = 1; o < kSortThreads; o <<= 1) {
            const int32_t v = tid >= o ? wsum[tid - o] : 0;
            __syncthreads();
            wsum[tid] += v;
            __syncthreads();
        }
        int32_t base = wsum[tid] - run;
        for (int q = 0; q < 16; ++q) { const int32_t c = cnt[tid * 16 + q]; cnt[tid * 16 + q] = base; base += c; }
        __syncthreads();
        for (int i = lo; i < hi; ++i) {
            const int p = cnt[((src[i] >> shift) & 15u) * kSortThreads + tid]++;
            t0[p] = k0[i]; t1[p] = k1[i]; t2[p] = k2[i];
        }
        __syncthreads();
        for (int i = tid; i < n; i += kSortThreads) { k0[i] = t0[i]; k1[i] = t1[i]; k2[i] = t2[i]; }
        __syncthreads();
    }
    for (int i = tid; i < n; i += kSortThreads) perm[b + i] = (int32_t)k0[i];
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// The sort proper on caller-provided scratch: cnt and cursor [n_seg + 1],
// err [1].  The scratch is cleared with a fill kernel (no memset node), and
// nothing here waits for the device.
static int enqueue_segsort(int n, int n_seg, const int32_t *seg, const float *pos, const int32_t *seq,
                           int32_t *perm, int32_t *seg_off, int32_t *cnt, int32_t *cursor, int32_t *err,
                           hipStream_t st)
{
    const int64_t nc = (int64_t)n_seg + 1;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, cnt, nc, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, err, (int64_t)1, 0);
    if (n > 0) hipLaunchKernelGGL(k_seg_hist, dim3((n + 255) / 256), dim3(256), 0, st, n, seg, cnt);
    hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(1024), 0, st, n_seg, cnt, seg_off, cursor);
    if (n > 0) hipLaunchKernelGGL(k_seg_scatter, dim3((n + 255) / 256), dim3(256), 0, st, n, seg, cursor, perm);
    hipLaunchKernelGGL(k_seg_lds_sort, dim3(n_seg), dim3(kSortThreads), 0, st, seg_off, pos, seq, perm, err);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

static int read_sort_flag(const int32_t *err, hipStream_t st)
{
    int32_t e = 0;
    if (hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, st) != hipSuccess) return -1;
    if (hipStreamSynchronize(st) != hipSuccess) return -1;
    return e ? 1 : 0;
}

int launch_segsort(int n, int n_seg, const int32_t *seg, const float *pos, const int32_t *seq, int32_t *perm,
                   int32_t *seg_off, int32_t *scratch, hipStream_t st)
{
    int32_t *cnt = scratch, *cursor = scratch + (n_seg + 1), *err = scratch + 2 * (n_seg + 1);
    if (enqueue_segsort(n, n_seg, seg, pos, seq, perm, seg_off, cnt, cursor, err, st) != 0) return -1;
    return read_sort_flag(err, st);
}

// ---------------------------------------------------------------------------
// Allocation-free segmented sort: its counters live in one fixed device
// array per GPU instead of a per-call allocation.  The array's name is only
// a host-side stand-in; its device address comes from hipGetSymbolAddress,
// taken once per device with that device current (segsort_scratch_init,
// called when a handle is created) and used for every launch and copy.
// ---------------------------------------------------------------------------
static __device__ __align__(256) int32_t scratch[2 * (kNoAllocMaxSegments + 1) + 64];

namespace {
std::mutex g_scratch_mu;
int32_t *g_scratch_ptr[kMaxDevices] = {};
}

int segsort_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return -1;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return 0;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) return -1;
    int32_t *p = nullptr;
    if (hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
    g_scratch_ptr[device] = p;
    return 0;
}

int launch_segsort_noalloc(int device, int n, int n_seg, const int32_t *seg, const float *pos, const int32_t *seq,
                           int32_t *perm, int32_t *seg_off, int32_t *status, hipStream_t st)
{
    if (n_seg < 1 || n_seg > kNoAllocMaxSegments) return -2;
    int32_t *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (device >= 0 && device < kMaxDevices) base = g_scratch_ptr[device];
    }
    if (!base) return -1;
    int32_t *cnt = base, *cursor = base + (n_seg + 1), *flag = base + 2 * (kNoAllocMaxSegments + 1);
    int32_t *err = status ? status : flag;
    if (enqueue_segsort(n, n_seg, seg, pos, seq, perm, seg_off, cnt, cursor, err, st) != 0) return -1;
    return status ? 0 : read_sort_flag(err, st);
}

// ---------------------------------------------------------------------------
// Optimisation loop (calibration and control, Methods "Optimization"): the
// count loss with its cotangent, and the AdamW update of one parameter group.
// ---------------------------------------------------------------------------

// One workgroup.  kind 0: mean over the n = det x nb counts of (q - y)^2,
// cotangent 2 (q - y) / n.  kind 1: (sum over the bins of detector det of q
// - target)^2, cotangent 2 (sum - target) on those bins, 0 elsewhere.  Fixed
// reduction order, so the loss is reproducible.
__global__ __launch_bounds__(1024) void k_count_loss(int n, int nb, const float *q, const float *y, int kind,
                                                      int det, double target, double *loss, float *gq)
{
    __shared__ double part[1024];
    const int tid = threadIdx.x;
    double acc = 0.0;
    if (kind == 0) {
        for (int i = tid; i < n; i += 1024) {
            const double e = (double)q[i] - (double)y[i];
            acc += e * e;
            gq[i] = (float)(2.0 * e / (double)n);
        }
    } else {
        for (int i = tid; i < n; i += 1024) gq[i] = 0.0f;
        if (tid < nb) acc = (double)q[(int64_t)det * nb + tid];
    }
    part[tid] = acc;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (tid < o) part[tid] += part[tid + o];
        __syncthreads();
    }
    if (kind == 0) {
        if (tid == 0) *loss = n > 0 ? part[0] / (double)n : 0.0;
    } else {
        const double e = part[0] - target;
        if (tid == 0) *loss = e * e;
        if (tid < nb) gq[(int64_t)det * nb + tid] = (float)(2.0 * e);
    }
}

// AdamW (Loshchilov and Hutter, decoupled weight decay) on float parameters
// in the coordinates x = (p - x0) / sc (x0 = 0, sc = 1: the parameters
// themselves), update t >= 1 with the gradient gx = g sc:
// m <- b1 m + (1 - b1) gx, v <- b2 v + (1 - b2) gx^2,
// x <- x - lr (m / (1 - b1^t) / (sqrt(v / (1 - b2^t)) + eps) + wd x),
// p = x0 + sc x, then the box [lo, min(hi, hi_vec[i])].  Arithmetic in double.
__global__ void k_adamw(int64_t n, float *p, const float *g, float *m, float *v, int t, double lr, double b1,
                        double b2, double eps, double wd, double x0, double sc, double lo, double hi,
                        const float *hi_vec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double gi = (double)g[i] * sc;
    const double mi = b1 * (double)m[i] + (1.0 - b1) * gi;
    const double vi = b2 * (double)v[i] + (1.0 - b2) * gi * gi;
    m[i] = (float)mi;
    v[i] = (float)vi;
    const double mh = mi / (1.0 - pow(b1, (double)t));
    const double vh = vi / (1.0 - pow(b2, (double)t));
    double x = ((double)p[i] - x0) / sc;
    x = x - lr * (mh / (sqrt(vh) + eps) + wd * x);
    double y = x0 + sc * x;
    double top = hi;
    if (hi_vec) top = fmin(top, (double)hi_vec[i]);
    y = fmin(fmax(y, lo), top);
    p[i] = (float)y;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_count_loss(int n, int nb, const float *q, const float *y, int kind, int det, double target,
                       double *loss, float *gq, hipStream_t st)
{
    hipLaunchKernelGGL(k_count_loss, dim3(1), dim3(1024), 0, st, n, nb, q, y, kind, det, target, loss, gq);
}

void launch_adamw(int64_t n, float *p, const float *g, float *m, float *v, int t, double lr, double b1, double b2,
                  double eps, double wd, double x0, double sc, double lo, double hi, const float *hi_vec,
                  hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_adamw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, p, g, m, v, t, lr, b1, b2,
                       eps, wd, x0, sc, lo, hi, hi_vec);
}
static inline int blocks_for(int64_t waves) { return (int)((waves + kWavesPerBlock - 1) / kWavesPerBlock); }

// one wavefront per launch record (offset, waves): first start and last end over its waves
__global__ __launch_bounds__(256) void k_stamp_reduce(const int64_t *off, const int32_t *waves, int n,
                                                      const unsigned long long *st, unsigned long long *out)
{
    const int r = (int)blockIdx.x * kWavesPerBlock + ((int)threadIdx.x >> 6), lane = (int)threadIdx.x & 63;
    if (r >= n) return;
    const unsigned long long *p = st + 2 * off[r];
    unsigned long long lo = ~0ull, hi = 0ull;
    for (int w = lane; w < waves[r]; w += 64) {
        lo = min(lo, p[2 * w]);
        hi = max(hi, p[2 * w + 1]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, (unsigned long long)__shfl_xor(lo, o));
        hi = max(hi, (unsigned long long)__shfl_xor(hi, o));
    }
    if (lane == 0) { out[2 * r] = lo; out[2 * r + 1] = hi; }
}
void launch_stamp_reduce(const int64_t *off, const int32_t *waves, int n, const unsigned long long *st,
                         unsigned long long *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_stamp_reduce, dim3((n + kWavesPerBlock - 1) / kWavesPerBlock), dim3(256), 0, s, off, waves,
                       n, st, out);
}

int link_blocks(const Dev &d)
{
    return std::max(1, ring_blocks(d, d.g_link));
}
int node_blocks(const Dev &d)
{
    return std::max(1, node_role_blocks(d.S * d.nd_n[0], 8, false) + node_role_blocks(d.S * d.nd_n[1], 16, false) +
                       node_role_blocks(d.S * d.nd_n[2], 32, false) + node_role_blocks(d.S * d.nd_n[3], 64, true));
}
int reverse_blocks(const Dev &d)
{
    return std::max(1, ring_blocks(d, d.g_rev));
}

template <typename K, typename... A>
static void launch(K kernel, int blocks, hipStream_t st, A... args)
{
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(256), 0, st, args...);
}

template <bool TAPE>
static void launch_link_t(const Dev &d, int t, int sample_b, int tape_k, hipStream_t st)
{
    switch (d.g_link) {
    case 8: launch(k_link<8, TAPE>, link_blocks(d), st, d, t, sample_b, tape_k); break;
    case 16: launch(k_link<16, TAPE>, link_blocks(d), st, d, t, sample_b, tape_k); break;
    case 32: launch(k_link<32, TAPE>, link_blocks(d), st, d, t, sample_b, tape_k); break;
    default: launch(k_link<64, TAPE>, link_blocks(d), st, d, t, sample_b, tape_k); break;
    }
}
void launch_link(const Dev &d, int t, int sample_b, int tape_k, hipStream_t st)
{
    if (tape_k >= 0) launch_link_t<true>(d, t, sample_b, tape_k, st);
    else launch_link_t<false>(d, t, sample_b, tape_k, st);
}
void launch_node(const Dev &d, int t, int tape_k, hipStream_t st)
{
    const int blocks = node_role_blocks(d.S * d.nd_n[0], 8, false) + node_role_blocks(d.S * d.nd_n[1], 16, false) +
                       node_role_blocks(d.S * d.nd_n[2], 32, false) + node_role_blocks(d.S * d.nd_n[3], 64, true);
    launch(k_node, std::max(blocks, 1), st, d, t, tape_k);
}
void launch_copy_multi(const CopyJobs &jobs, hipStream_t st)
{
    uint64_t total = 0;
    for (int k = 0; k < jobs.n; ++k) total += jobs.job[k].bytes / 16;
    const uint64_t want = (total + 255) / 256;
    const int blocks = (int)std::max<uint64_t>(1, std::min<uint64_t>(want, 2048));
    hipLaunchKernelGGL(k_copy_multi, dim3(blocks), dim3(256), 0, st, jobs);
}
void launch_tape_snapshot(const Dev &d, int tape_k, hipStream_t st)
{
    hipLaunchKernelGGL(k_tape_snapshot, dim3(blocks_for((int64_t)d.S * d.L)), dim3(256), 0, st, d, tape_k);
}
void launch_reverse(const Dev &d, int t, int tape_k, int init, hipStream_t st)
{
    switch (d.g_rev) {
    case 8: launch(k_reverse<8>, reverse_blocks(d), st, d, t, tape_k, init); break;
    case 16: launch(k_reverse<16>, reverse_blocks(d), st, d, t, tape_k, init); break;
    case 32: launch(k_reverse<32>, reverse_blocks(d), st, d, t, tape_k, init); break;
    default: launch(k_reverse<64>, reverse_blocks(d), st, d, t, tape_k, init); break;
    }
}
void launch_ste(const Dev &d, int t, int tape_k, hipStream_t st)
{
    launch(k_ste, std::max(node_blocks(d), 1), st, d, t, tape_k);
}
void launch_theta_sum(const Dev &d, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_theta_sum, dim3(d.S), dim3(64), 0, st, d, out);
}
void launch_rate_grad(const Dev &d, float *g, hipStream_t st)
{
    if ((int64_t)d.S * d.O == 0) return;
    hipLaunchKernelGGL(k_rate_grad, dim3(blocks_for((int64_t)d.S * d.O)), dim3(256), 0, st, d, g);
}
void launch_derive(const Dev &d, const float *cap_mult, const float *capacity, const float *beta,
                   const float *cost, double *util, double *acc, float *vfree, float *spacing, LinkNd *lnd,
                   LinkCf *lcf, RevCf *rcf, hipStream_t st)
{
    const int64_t n = (int64_t)d.S * d.L;
    hipLaunchKernelGGL(k_derive, dim3((int)((n + 255) / 256)), dim3(256), 0, st, d, cap_mult, capacity, beta, cost,
                       util, acc, vfree, spacing, lnd, lcf, rcf);
}
void launch_ttt(const Dev &d, int T, double *out, int64_t *vsteps, unsigned long long *acc, hipStream_t st)
{
    // acc: 2 x S zeroed here with a fill kernel (no memset node, so the sequence can sit in a graph)
    hipLaunchKernelGGL(k_zero_u64, dim3((2 * d.S + 255) / 256), dim3(256), 0, st, acc, 2 * d.S);
    const int nb = std::max(1, std::min(1024, (d.N + 2047) / 2048));
    hipLaunchKernelGGL(k_ttt, dim3(nb, d.S), dim3(256), 0, st, d, T, acc);
    hipLaunchKernelGGL(k_ttt_final, dim3((d.S + 255) / 256), dim3(256), 0, st, d.S, d.dt, acc, out, vsteps);
}
void launch_counts(const Dev &d, float *out, hipStream_t st)
{
    const int64_t n = (int64_t)d.S * d.D * d.nb;
    if (n == 0) return;
    hipLaunchKernelGGL(k_counts, dim3((int)((n + 255) / 256)), dim3(256), 0, st, d, out);
}
void launch_gather_links(const double *src, const int32_t *linv, float *dst, int S, int L, hipStream_t st)
{
    const int64_t n = (int64_t)S * L;
    if (n == 0) return;
    hipLaunchKernelGGL(k_gather_links, dim3((int)((n + 255) / 256)), dim3(256), 0, st, src, linv, dst, S, L);
}
void launch_d2f(const double *src, float *dst, int64_t n, hipStream_t st)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_d2f, dim3((int)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
}
__global__ void k_gumbel_fast(int n, const uint32_t *w, float *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = gumbel_fast(w[i]);
}
void launch_gumbel_fast(int n, const uint32_t *w, float *out, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gumbel_fast, dim3((n + 255) / 256), dim3(256), 0, st, n, w, out);
}
void launch_philox(int n, const uint32_t *ctr, const uint32_t *key, uint32_t *out, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_philox, dim3((n + 255) / 256), dim3(256), 0, st, n, ctr, key, out);
}

}  // namespace sim
