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

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

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

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the Weyl key schedule.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
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

// Route choice (SI-B): candidates are the out-links of node v that can still
// reach the destination (and are not the reverse of `from` unless U-turns
// are allowed); utility beta/c - theta*(t_ff + shortest time from the link's
// head), hard choice argmax(V + g) (Gumbel-max; the temperature only shapes
// the gradient).  Ties go to the lower candidate index.
__device__ int choose_link(const Dev &d, int s, int a, int v, int from, int t, int *ties)
{
    const int beg = d.out_off[v], end = d.out_off[v + 1];
    const double *dist = d.dist + (int64_t)d.agent_didx[a] * d.Nn;
    const uint64_t seed = d.seed[s];
    double best = -INFINITY, second = -INFINITY;
    int arg = CH_STUCK, blk = -1;
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    for (int k = beg; k < end; ++k) {
        const int m = d.out_lnk[k], c = k - beg;
        if (!d.allow_uturn && from >= 0 && d.head[m] == d.tail[from]) continue;
        const double dm = dist[d.head[m]];
        if (!(dm < INFINITY)) continue;
        if ((c >> 2) != blk) { blk = c >> 2; draw4(seed, a, t, 0, blk, w); }
        const double V = d.util[(int64_t)s * d.L + m] - d.theta * (d.tff[m] + dm);
        const double sc = V + gumbel_of(w[c & 3]);
        if (sc > best) { second = best; best = sc; arg = m; }
        else if (sc > second) second = sc;
    }
    if (arg >= 0 && second > -INFINITY && best - second < 1e-12 * (1.0 + fabs(best))) ++*ties;
    return arg;
}

__device__ __forceinline__ double merge_noise(uint64_t seed, int a, int t)
{
    uint32_t w[4];
    draw4(seed, a, t, 1, 0, w);
    return gumbel_of(w[0]);
}

// ---------------------------------------------------------------------------
// Link phase: per (scenario, link) segment, in place on the ring.
//   Newell car-following with the link cap (Methods eq. newell_model; SI-A),
//   position form x' = min(x + u dt, max(x, x_lead - dn/kappa)), x_hat =
//   min(x', L); leader = rank - lanes; arrival (x_hat >= L - 0.01), vacancy
//   (entry slots = lanes - #(x_hat <= dn/kappa)), token accrual, detector
//   crossings, order check, and the route choice of the heads.
// Chunks of 64 ranks are processed back to front so every leader is read
// before its own update is written (all inputs are time-t positions).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_link(Dev d, int t, int sample_b, int tape_k)
{
    const int lane = lane_id();
    const int seg = xcd_tile() * kWavesPerBlock + (threadIdx.x >> 6);
    if (seg >= d.S * d.L) return;
    const int s = seg / d.L, j = seg - s * d.L;
    const int h0 = d.rhead[seg], n = d.rtail[seg] - h0;
    const int cap = d.cap[j], ln = d.lanes[j];
    const int64_t base = (int64_t)s * d.ring_total + d.ring_base[j];
    const float vf = d.vfree[seg], sp = d.spacing[seg], Lj = d.length[j], thr = d.thr[j];
    const int d0 = d.det_off[j], nd = d.det_off[j + 1] - d0;
    int64_t tb = -1;
    if (tape_k >= 0) {
        tb = (int64_t)tape_k * d.S * d.ring_total + base;
        if (lane == 0) {
            d.tape_head[(int64_t)tape_k * d.S * d.L + seg] = h0;
            d.tape_tail[(int64_t)tape_k * d.S * d.L + seg] = h0 + n;
        }
    }
    if (lane == 0 && n > cap) atomicOr(&d.err[ERR_RING_OVERFLOW], 1);

    int nh = 0, nocc = 0, viol = 0;
    int dcnt[kMaxDetPerLink] = {0, 0, 0, 0};
    float dpos[kMaxDetPerLink];
    for (int k = 0; k < kMaxDetPerLink; ++k) dpos[k] = k < nd ? d.det_pos[d.det_list[d0 + k]] : 0.f;
    float next_first = INFINITY;   // x_hat of rank 64(c+1), the chunk processed before
    bool have_next = false;
    for (int c = (n - 1) >> 6; c >= 0; --c) {
        const int r = (c << 6) + lane;
        const bool v = r < n;
        float x = 0.f, xl = 0.f;
        int slot = 0;
        if (v) {
            slot = (h0 + r) % cap;
            x = d.ring_pos[base + slot];
            if (r >= ln) xl = d.ring_pos[base + (h0 + r - ln) % cap];
            if (tb >= 0) {
                d.tape_pos[tb + slot] = x;
                d.tape_agent[tb + slot] = d.ring_agent[base + slot];
            }
        }
        const float xf = x + vf;
        float xn = xf;
        if (r >= ln) {
            const float xc = xl - sp;
            const float cc = (x > xc) ? x : xc;
            xn = (xf <= cc) ? xf : cc;
        }
        const float xh = (xn > Lj) ? Lj : xn;
        if (v) d.ring_pos[base + slot] = xh;
        nh += __popcll(__ballot(v && xh >= thr));
        nocc += __popcll(__ballot(v && xh <= sp));
#pragma unroll
        for (int k = 0; k < kMaxDetPerLink; ++k)
            if (k < nd) dcnt[k] += __popcll(__ballot(v && xh >= dpos[k]));
        // order check (rank r-1 must not be behind rank r)
        const float up = __shfl_up(xh, 1);
        bool bad = v && lane > 0 && up < xh;
        if (v && lane == 63 && have_next && xh < next_first) bad = true;
        viol += __popcll(__ballot(bad));
        next_first = __shfl(xh, 0);
        have_next = true;
    }
    const int h = min(nh, min(ln, d.maxl));
    if (lane == 0) {
        d.B[seg] += d.acc[seg];
        d.slots[seg] = max(0, ln - nocc);
        d.nheads[seg] = h;
        if (viol) atomicAdd((unsigned long long *)&d.ctr[s * CTR_N + CTR_ORDER_VIOL], (unsigned long long)viol);
        if (sample_b >= 0) {
            const int64_t E = d.E[seg];
            for (int k = 0; k < nd; ++k)
                d.cum[((int64_t)s * d.D + d.det_list[d0 + k]) * d.nb + sample_b] = (int32_t)(E + dcnt[k]);
        }
    }
    // heads: route choice and merge key
    int ties = 0;
    if (lane < h) {
        const int a = d.ring_agent[base + (h0 + lane) % cap];
        const int vnode = d.head[j];
        int ch;
        if (d.agent_dest[a] == vnode) ch = CH_EXIT;
        else ch = choose_link(d, s, a, vnode, j, t, &ties);
        const int64_t hi = (int64_t)seg * d.maxl + lane;
        d.head_agent[hi] = a;
        d.head_choice[hi] = ch;
        d.head_key[hi] = (double)d.alpha[seg] + merge_noise(d.seed[s], a, t);
    }
    if (ties) atomicAdd((unsigned long long *)&d.ctr[s * CTR_N + CTR_TIES], (unsigned long long)ties);
}

// ---------------------------------------------------------------------------
// Node phase: per (scenario, node), one wavefront.
//   Releases into the node's origin queues, the origin fronts' route choice,
//   merge choice per out-link (top-k by alpha_from + Gumbel, k = entry slots;
//   SI-B merge choice), FIFO resolve of each in-link's heads against its
//   token bucket, and the grafted transfer: leavers pop from the in-link
//   ring, entrants push at position 0 onto the out-link ring (SI-B eq.
//   transfer; the graft itself lives in the adjoint).
// Candidate lanes: in-link q, head rank r -> lane q*maxl + r; then origins.
// All cross-lane traffic goes through readlane/shuffles.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_node(Dev d, int t)
{
    const int lane = lane_id();
    const int wid = xcd_tile() * kWavesPerBlock + (threadIdx.x >> 6);
    if (wid >= d.S * d.Nn) return;
    const int s = wid / d.Nn, v = wid - s * d.Nn;
    const int maxl = d.maxl;
    const int i0 = d.in_off[v], deg = d.in_off[v + 1] - i0;
    const int o0 = d.org_off[v], norg = d.org_off[v + 1] - o0;
    const int nc = deg * maxl + norg;
    const int oo = d.out_off[v], dego = d.out_off[v + 1] - oo;
    const uint64_t seed = d.seed[s];
    int ties = 0;

    // ---- candidate of this lane ----
    int ch = CH_NONE, ag = -1;
    double key = 0.0;
    int origin = -1;
    if (lane < deg * maxl) {
        const int q = lane / maxl, r = lane - q * maxl;
        const int sj = s * d.L + d.in_lnk[i0 + q];
        if (r < d.nheads[sj]) {
            const int64_t hi = (int64_t)sj * maxl + r;
            ag = d.head_agent[hi];
            ch = d.head_choice[hi];
            key = d.head_key[hi];
        }
    } else if (lane < nc) {
        origin = d.org_list[o0 + lane - deg * maxl];
        const int so = s * d.O + origin;
        const int qb = d.q_off[origin], qn = d.q_off[origin + 1] - qb;
        // release (serial per origin; a handful of agents per step)
        int rel = d.rel_ptr[so], newrel = rel;
        if (d.fixed_mode) {
            while (newrel < qn && d.q_rstep[qb + newrel] <= (int64_t)t) {
                const int a = d.q_list[qb + newrel];
                d.status[(int64_t)s * d.N + a] = AG_QUEUED;
                d.rel_t[(int64_t)s * d.N + a] = t;
                ++newrel;
            }
        } else {
            double inc = 0.0;
            const double t0 = t * d.dt, t1 = (t + 1) * d.dt;
            for (int b = 0; b < d.n_rate_bins; ++b) {
                const double lo = fmax(b * d.rate_bin_s, t0), hi = fmin((b + 1) * d.rate_bin_s, t1);
                if (hi > lo) inc += (double)d.rates[((int64_t)s * d.O + origin) * d.n_rate_bins + b] * (hi - lo);
            }
            const double D = d.Dacc[so] + inc;
            d.Dacc[so] = D;
            const double r = inc / d.dt;
            while (newrel < qn && (double)(newrel + 1) <= D) {
                const int a = d.q_list[qb + newrel];
                const int64_t ga = (int64_t)s * d.N + a;
                d.status[ga] = AG_QUEUED;
                d.tstar[ga] = t1 - (D - (double)(newrel + 1)) / r;
                d.rel_t[ga] = t;
                ++newrel;
            }
        }
        if (newrel != rel) {
            d.rel_ptr[so] = newrel;
            atomicAdd((unsigned long long *)&d.ctr[s * CTR_N + CTR_RELEASED], (unsigned long long)(newrel - rel));
        }
        const int dp = d.dep_ptr[so];
        if (dp < newrel) {
            ag = d.q_list[qb + dp];
            ch = choose_link(d, s, ag, v, -1, t, &ties);
            key = 1.0 + merge_noise(seed, ag, t);
        }
    }
    if (nc > kWave) { if (lane == 0) atomicOr(&d.err[ERR_CAND_OVERFLOW], 1); return; }

    // ---- merge: rank among candidates wanting the same link ----
    int rank = 0, next_gap_tie = 0;
    for (int src = 0; src < nc; ++src) {
        const int c2 = readlane_i(ch, src);
        const double k2 = readlane_d(key, src);
        const int a2 = readlane_i(ag, src);
        if (ch >= 0 && c2 == ch && src != lane) {
            if (k2 > key || (k2 == key && a2 < ag)) ++rank;
            else if (key - k2 < 1e-12 * (1.0 + fabs(key))) next_gap_tie = 1;
        }
    }
    int won = 0;
    if (ch >= 0) won = rank < d.slots[s * d.L + ch];
    // one near-tie per candidate that has a close successor (as the oracle counts adjacent pairs)
    ties += (ch >= 0) ? next_gap_tie : 0;

    // ---- resolve: lane q < deg walks in-link q's heads in rank order ----
    int np = 0, stuck = 0;
    double Bj = 0.0;
    int sjq = -1, nhq = 0;
    if (lane < deg) {
        sjq = s * d.L + d.in_lnk[i0 + lane];
        Bj = d.B[sjq];
        nhq = d.nheads[sjq];
    }
    bool stop = false;
    for (int r = 0; r < maxl; ++r) {
        const int src = min(lane * maxl + r, kWave - 1);
        const int c2 = __shfl(ch, src);
        const int w2 = __shfl(won, src);
        if (lane < deg && !stop && r < nhq) {
            if (c2 == CH_EXIT) ++np;
            else if (c2 >= 0 && w2 && Bj >= 1.0) { Bj -= 1.0; ++np; }
            else { stop = true; if (c2 == CH_STUCK) ++stuck; }
        }
    }
    if (lane < deg) {
        d.B[sjq] = Bj > 1.0 ? 1.0 : Bj;
        if (np) {
            d.E[sjq] += np;
            d.rhead[sjq] += np;
        }
    }
    // did this lane's candidate pass?  (shuffles stay in uniform control flow)
    const int q_of_lane = (lane < deg * maxl) ? lane / maxl : 0;
    const int np_q = __shfl(np, q_of_lane);
    int passed = 0;
    if (lane < deg * maxl) passed = (ag >= 0) && (lane - q_of_lane * maxl) < np_q;
    else passed = (origin >= 0 && ag >= 0 && won);

    // ---- out-links: count entrants, advance ring tails ----
    const int my_m = (lane < dego) ? d.out_lnk[oo + lane] : -100;
    int tail_old = 0, nent = 0;
    if (lane < dego) tail_old = d.rtail[s * d.L + my_m];
    for (int src = 0; src < nc; ++src) {
        const int c2 = readlane_i(ch, src);
        const int p2 = readlane_i(passed, src);
        nent += (p2 && c2 == my_m);
    }
    if (lane < dego && nent) d.rtail[s * d.L + my_m] = tail_old + nent;
    // ---- entrants: position in key order among passed winners of the link ----
    int erank = 0;
    for (int src = 0; src < nc; ++src) {
        const int c2 = readlane_i(ch, src);
        const int p2 = readlane_i(passed, src);
        const double k2 = readlane_d(key, src);
        const int a2 = readlane_i(ag, src);
        if (passed && ch >= 0 && p2 && c2 == ch && src != lane && (k2 > key || (k2 == key && a2 < ag))) ++erank;
    }
    int oidx = 0;
    if (passed && ch >= 0)
        for (int k = 0; k < dego; ++k)
            if (d.out_lnk[oo + k] == ch) { oidx = k; break; }
    const int tbase = __shfl(tail_old, oidx);
    const int64_t ga = (int64_t)s * d.N + (ag >= 0 ? ag : 0);
    if (passed) {
        if (ch >= 0) {
            const int capm = d.cap[ch];
            const int64_t slot = (int64_t)s * d.ring_total + d.ring_base[ch] + (tbase + erank) % capm;
            d.ring_agent[slot] = ag;
            d.ring_pos[slot] = 0.f;
            if (origin >= 0) {
                d.status[ga] = AG_ON;
                d.dep_t[ga] = t;
                d.dep_ptr[s * d.O + origin] += 1;
            }
        } else {
            d.status[ga] = AG_EXITED;
            d.exit_t[ga] = t;
        }
    }
    // counters
    const int n_dep = __popcll(__ballot(passed && origin >= 0));
    const int n_exit = __popcll(__ballot(passed && ch == CH_EXIT));
    const int n_tr = __popcll(__ballot(passed && ch >= 0 && origin < 0));
    int tot_ties = ties, tot_stuck = stuck;
    for (int o = 32; o > 0; o >>= 1) { tot_ties += __shfl_xor(tot_ties, o); tot_stuck += __shfl_xor(tot_stuck, o); }
    if (lane == 0) {
        unsigned long long *c = (unsigned long long *)&d.ctr[s * CTR_N];
        if (n_dep) atomicAdd(c + CTR_DEPARTED, (unsigned long long)n_dep);
        if (n_exit) atomicAdd(c + CTR_EXITED, (unsigned long long)n_exit);
        if (n_tr) atomicAdd(c + CTR_TRANSFERS, (unsigned long long)n_tr);
        if (tot_ties) atomicAdd(c + CTR_TIES, (unsigned long long)tot_ties);
        if (tot_stuck) atomicAdd(c + CTR_STUCK, (unsigned long long)tot_stuck);
    }
}

// Tape entry without an update (the state at the end of a replay window).
__global__ __launch_bounds__(256) void k_tape_snapshot(Dev d, int tape_k)
{
    const int lane = lane_id();
    const int seg = xcd_tile() * kWavesPerBlock + (threadIdx.x >> 6);
    if (seg >= d.S * d.L) return;
    const int s = seg / d.L, j = seg - s * d.L;
    const int h0 = d.rhead[seg], n = d.rtail[seg] - h0, cap = d.cap[j];
    const int64_t base = (int64_t)s * d.ring_total + d.ring_base[j];
    const int64_t tb = (int64_t)tape_k * d.S * d.ring_total + base;
    if (lane == 0) {
        d.tape_head[(int64_t)tape_k * d.S * d.L + seg] = h0;
        d.tape_tail[(int64_t)tape_k * d.S * d.L + seg] = h0 + n;
    }
    for (int r = lane; r < n; r += kWave) {
        const int slot = (h0 + r) % cap;
        d.tape_pos[tb + slot] = d.ring_pos[base + slot];
        d.tape_agent[tb + slot] = d.ring_agent[base + slot];
    }
}

// ---------------------------------------------------------------------------
// Reverse of step t (tape entry k holds time t, k+1 time t+1), per segment.
// Input: adj[a] = dL/dx_a(t+1) for agents on the network at t+1 (sampled
// counts at t+1 already added).  Output: adj[a] = dL/dx_a(t) for agents on
// this link at t, plus the counts sampled at t and the departure grafts of
// agents that entered at t.  Branches are recomputed from the taped time-t
// positions with the forward's exact float operations.
//   cap (SI-A eq. tg): dx_hat/dx' = 1 in both branches;
//   transfer (SI-B eq. transfer, SI-C): the entry position carries x_hat;
//   exit: total travel time falls by (x_hat - sg x_hat)/u of the last link;
//   free: x' = x + u dt; congested: x' = x_lead - dn/kappa; stopped: x' = x.
// Each agent has at most one follower (rank + lanes), so the leader term is
// a gather: chunks go front to back so followers are read before they are
// overwritten.  init = 1: adj = dL/dx(T) at the final state (no step).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reverse(Dev d, int t, int tape_k, int init)
{
    const int lane = lane_id();
    const int seg = xcd_tile() * kWavesPerBlock + (threadIdx.x >> 6);
    if (seg >= d.S * d.L) return;
    const int s = seg / d.L, j = seg - s * d.L;
    const int64_t SL = (int64_t)d.S * d.L;
    const int hk = d.tape_head[tape_k * SL + seg];
    const int n = d.tape_tail[tape_k * SL + seg] - hk;
    const int npass = init ? 0 : d.tape_head[(tape_k + 1) * SL + seg] - hk;
    const int cap = d.cap[j], ln = d.lanes[j], vhead = d.head[j];
    const int64_t base = (int64_t)s * d.ring_total + d.ring_base[j];
    const int64_t tb = (int64_t)tape_k * d.S * d.ring_total + base;
    const float vf = d.vfree[seg], sp = d.spacing[seg], Lj = d.length[j];
    const float uj = d.u[seg], kap = d.kappa[seg];
    const double dkap = (double)d.platoon / ((double)kap * (double)kap);
    const double gTs = d.gT ? d.gT[s] : 0.0;
    const float exit_adj = (float)(-gTs / (double)uj);
    const int64_t sN = (int64_t)s * d.N;
    // counts sampled at time t
    int sb = -1;
    if (d.gQ && d.cbs > 0 && t > 0 && t % d.cbs == 0 && t / d.cbs <= d.nb) sb = t / d.cbs - 1;
    const int d0 = d.det_off[j], nd = d.det_off[j + 1] - d0;
    const float sc = 5.0f / Lj;
    double gu = 0.0, gk = 0.0;
    for (int c = 0; (c << 6) < n; ++c) {
        const int r = (c << 6) + lane;
        const bool v = r < n;
        float x = 0.f;
        int a = 0;
        if (v) {
            const int slot = (hk + r) % cap;
            x = d.tape_pos[tb + slot];
            a = d.tape_agent[tb + slot];
        }
        float anew = 0.f;
        if (!init) {
            // own branch
            int br = 0;  // 0 free, 1 congested, 2 stopped
            if (v && r >= ln) {
                const float xl = d.tape_pos[tb + (hk + r - ln) % cap];
                const float xf = x + vf, xc = xl - sp;
                const float cc = (x > xc) ? x : xc;
                br = (xf <= cc) ? 0 : ((x > xc) ? 2 : 1);
            }
            float ap = 0.f;
            if (v) ap = (r < npass && d.agent_dest[a] == vhead) ? exit_adj : d.adj[sN + a];
            // follower (rank r + lanes) in the congested branch passes its adjoint to us
            float af = 0.f;
            const int fr = r + ln;
            if (v && fr < n) {
                const int fs = (hk + fr) % cap;
                const float xfol = d.tape_pos[tb + fs];
                const float ff = xfol + vf, xc = x - sp;
                const float cc = (xfol > xc) ? xfol : xc;
                const bool cong = !(ff <= cc) && !(xfol > xc);
                if (cong) af = d.adj[sN + d.tape_agent[tb + fs]];
            }
            anew = (br != 1 ? ap : 0.f) + af;
            if (v && br == 0) gu += d.dt * (double)ap;
            if (v && br == 1) gk += dkap * (double)ap;
        } else if (v && d.gx) {
            anew = d.gx[sN + a];
        }
        if (sb >= 0 && v) {
            for (int k = 0; k < nd; ++k) {
                const int det = d.det_list[d0 + k];
                const int64_t qi = ((int64_t)s * d.D + det) * d.nb;
                const float gC = d.gQ[qi + sb] - (sb + 1 < d.nb ? d.gQ[qi + sb + 1] : 0.f);
                const float z = sc * (x - d.det_pos[det]);
                const float sg = 1.0f / (1.0f + expf(-z));
                anew += gC * sc * sg * (1.0f - sg);
            }
        }
        if (v) {
            d.adj[sN + a] = anew;
            if (d.dep_t[sN + a] == t - 1) d.depg[sN + a] = anew * uj;
        }
    }
    gu = wave_sum_d(gu);
    gk = wave_sum_d(gk);
    if (lane == 0 && !init) {
        d.gu[seg] += gu;
        d.gk[seg] += gk;
    }
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
    for (int b0 = 0; b0 < nbins; b0 += kWave) {
        const int b = b0 + lane;
        double acc = 0.0;
        const double lo = b * d.rate_bin_s, hi = (b + 1) * d.rate_bin_s;
        for (int k = 0; k < qn; ++k) {
            const int a = d.q_list[qb + k];
            if (d.dep_t[sN + a] < 0) continue;
            const double ts = d.tstar[sN + a];
            const int rb = min(nbins - 1, max(0, (int)floor((double)d.rel_t[sN + a] * d.dt / d.rate_bin_s)));
            const double ov = fmin(hi, ts) - lo;
            if (b < nbins && ov > 0) acc += (double)d.depg[sN + a] * ov / (double)rates[rb];
        }
        if (b < nbins) g[((int64_t)s * d.O + o) * nbins + b] = (float)acc;
    }
}

// Derived per-(scenario, link) constants.
__global__ void k_derive(Dev d, const float *cap_mult, const float *capacity, const float *beta,
                         const float *cost, double *util, double *acc, float *vfree, float *spacing)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)d.S * d.L) return;
    const int j = (int)(i % d.L);
    vfree[i] = __fmul_rn(d.u[i], (float)d.dt);
    spacing[i] = __fdiv_rn((float)d.platoon, d.kappa[i]);
    util[i] = (double)beta[i] / (double)cost[i];
    acc[i] = (double)cap_mult[i] * (double)capacity[j] * (double)d.lanes[j] * d.dt;
}

// Total travel time and vehicle-steps per scenario: dt * sum over released
// agents of ((exit step or T) - release step), i.e. agent-steps spent queued
// or on the network after each step, and sum over departed agents of
// ((exit step or T) - departure step), the agent-steps on the network.  One
// workgroup per scenario, fixed reduction order.
__global__ __launch_bounds__(256) void k_ttt(Dev d, int T, double *out, int64_t *vsteps)
{
    __shared__ double part[256];
    __shared__ long long vpart[256];
    const int s = blockIdx.x;
    const int64_t sN = (int64_t)s * d.N;
    double acc = 0.0;
    long long vs = 0;
    for (int i = threadIdx.x; i < d.N; i += 256) {
        const uint8_t st = d.status[sN + i];
        if (st == AG_WAIT) continue;
        const int e = (st == AG_EXITED) ? d.exit_t[sN + i] : T;
        acc += (double)(e - d.rel_t[sN + i]);
        if (st != AG_QUEUED) vs += e - (d.dep_t[sN + i] >= 0 ? d.dep_t[sN + i] : 0);  // placed agents: from t = 0
    }
    part[threadIdx.x] = acc;
    vpart[threadIdx.x] = vs;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) { part[threadIdx.x] += part[threadIdx.x + o]; vpart[threadIdx.x] += vpart[threadIdx.x + o]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out[s] = part[0] * d.dt; if (vsteps) vsteps[s] = vpart[0]; }
}

// Interval counts from cumulative samples.
__global__ void k_counts(Dev d, float *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)d.S * d.D * d.nb) return;
    const int b = (int)(i % d.nb);
    out[i] = (float)(d.cum[i] - (b > 0 ? d.cum[i - 1] : 0));
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

int launch_segsort(int n, int n_seg, const int32_t *seg, const float *pos, const int32_t *seq, int32_t *perm,
                   int32_t *seg_off, int32_t *scratch, hipStream_t st)
{
    int32_t *cnt = scratch, *cursor = scratch + (n_seg + 1), *err = scratch + 2 * (n_seg + 1);
    if (hipMemsetAsync(scratch, 0, ((size_t)2 * (n_seg + 1) + 1) * 4, st) != hipSuccess) return -1;
    if (n > 0) hipLaunchKernelGGL(k_seg_hist, dim3((n + 255) / 256), dim3(256), 0, st, n, seg, cnt);
    hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(1024), 0, st, n_seg, cnt, seg_off, cursor);
    if (n > 0) hipLaunchKernelGGL(k_seg_scatter, dim3((n + 255) / 256), dim3(256), 0, st, n, seg, cursor, perm);
    hipLaunchKernelGGL(k_seg_lds_sort, dim3(n_seg), dim3(kSortThreads), 0, st, seg_off, pos, seq, perm, err);
    int32_t e = 0;
    if (hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, st) != hipSuccess) return -1;
    if (hipStreamSynchronize(st) != hipSuccess) return -1;
    return e ? 1 : 0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int blocks_for(int64_t waves) { return (int)((waves + kWavesPerBlock - 1) / kWavesPerBlock); }

void launch_link(const Dev &d, int t, int sample_b, int tape_k, hipStream_t st)
{
    hipLaunchKernelGGL(k_link, dim3(blocks_for((int64_t)d.S * d.L)), dim3(256), 0, st, d, t, sample_b, tape_k);
}
void launch_node(const Dev &d, int t, hipStream_t st)
{
    hipLaunchKernelGGL(k_node, dim3(blocks_for((int64_t)d.S * d.Nn)), dim3(256), 0, st, d, t);
}
void launch_tape_snapshot(const Dev &d, int tape_k, hipStream_t st)
{
    hipLaunchKernelGGL(k_tape_snapshot, dim3(blocks_for((int64_t)d.S * d.L)), dim3(256), 0, st, d, tape_k);
}
void launch_reverse(const Dev &d, int t, int tape_k, int init, hipStream_t st)
{
    hipLaunchKernelGGL(k_reverse, dim3(blocks_for((int64_t)d.S * d.L)), dim3(256), 0, st, d, t, tape_k, init);
}
void launch_rate_grad(const Dev &d, float *g, hipStream_t st)
{
    hipLaunchKernelGGL(k_rate_grad, dim3(blocks_for((int64_t)d.S * d.O)), dim3(256), 0, st, d, g);
}
void launch_derive(const Dev &d, const float *cap_mult, const float *capacity, const float *beta,
                   const float *cost, double *util, double *acc, float *vfree, float *spacing, hipStream_t st)
{
    const int64_t n = (int64_t)d.S * d.L;
    hipLaunchKernelGGL(k_derive, dim3((int)((n + 255) / 256)), dim3(256), 0, st, d, cap_mult, capacity, beta, cost,
                       util, acc, vfree, spacing);
}
void launch_ttt(const Dev &d, int T, double *out, int64_t *vsteps, hipStream_t st)
{
    hipLaunchKernelGGL(k_ttt, dim3(d.S), dim3(256), 0, st, d, T, out, vsteps);
}
void launch_counts(const Dev &d, float *out, hipStream_t st)
{
    const int64_t n = (int64_t)d.S * d.D * d.nb;
    if (n == 0) return;
    hipLaunchKernelGGL(k_counts, dim3((int)((n + 255) / 256)), dim3(256), 0, st, d, out);
}
void launch_d2f(const double *src, float *dst, int64_t n, hipStream_t st)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_d2f, dim3((int)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
}
void launch_philox(int n, const uint32_t *ctr, const uint32_t *key, uint32_t *out, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_philox, dim3((n + 255) / 256), dim3(256), 0, st, n, ctr, key, out);
}

}  // namespace sim
