// Algorithm 1 steps other than evaluation: sampling (1), selection (3),
// log-rank weights (4), mean (5) and covariance (6) updates, the Cholesky
// factor used for sampling, and the gradient polish of the elites.
// All state lives on the device; no step needs the host, so the loop can be
// captured into a graph.  Reductions run in a fixed order (deterministic).
#include "launch.h"

namespace cp {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and Box-Muller normals
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
        const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

__device__ __forceinline__ double uniform01(uint32_t x) {
    return (2.0 * (double)(x >> 9) + 1.0) * (1.0 / 16777216.0);
}

__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double &z0, double &z1) {
    const double two_pi = 6.283185307179586476925286766559;
    const double r = sqrt(-2.0 * log(uniform01(a)));
    const double th = two_pi * uniform01(b);
    z0 = r * cos(th);
    z1 = r * sin(th);
}

// ---------------------------------------------------------------------------
// state initialisation: mu_0 evenly spaced on the start-goal segment,
// C_0 = sigma0^2 I, log-rank weights
// ---------------------------------------------------------------------------

__global__ void k_init_state(PlanView P, OptView O, float sigma0) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int D = O.D;
    if (tid < D) {
        const int k = tid / O.n_act, a = tid % O.n_act;
        const int jj = O.act[a];
        const double qs = P.qs[jj], qg = P.qg[jj];
        O.mu[tid] = qs + (double)(k + 1) / (double)(P.K + 1) * (qg - qs);
    }
    for (int i = tid; i < D * D; i += gridDim.x * blockDim.x) {
        const double s = (double)sigma0;
        O.C[i] = (i / D == i % D) ? s * s : 0.0;
    }
    if (tid == 0) {
        // w_j = (ln(nu + 1/2) - ln j) / sum_k (ln(nu + 1/2) - ln k), summed in rank order
        const double lmax = log((double)O.nu + 0.5);
        double s = 0.0;
        for (int j = 1; j <= O.nu; ++j) s += lmax - log((double)j);
        for (int j = 1; j <= O.nu; ++j) O.w[j - 1] = (lmax - log((double)j)) / s;
        *O.t = 0;
        *O.status = 0;
        *O.best_cost = kInf;
    }
}

// ---------------------------------------------------------------------------
// sampling: xi_b = mu + L z_b (double), waypoints W_b (float)
// ---------------------------------------------------------------------------

constexpr int kSampleTile = 16;  // paths per block

__device__ __forceinline__ void sample_body(const PlanView &P, const OptView &O, int tile) {
    __shared__ double z[kSampleTile][CP_MAX_DIM + 1];  // padded rows: lanes of one column read across paths
    __shared__ int wofs[CP_MAX_DIM];                   // coordinate e -> its offset in a path's waypoints
    const int D = O.D, n = P.n_joints, per = P.K * n;
    const int b0 = tile * kSampleTile;
    const uint32_t t = (uint32_t)*O.t;
    const uint32_t k0 = (uint32_t)O.seed, k1 = (uint32_t)(O.seed >> 32);
    const int G = (D + 3) / 4;
    // items run path-minor (bl = idx mod 16): no division by a runtime count
    for (int idx = threadIdx.x; idx < kSampleTile * G; idx += blockDim.x) {
        const int bl = idx % kSampleTile, g = idx / kSampleTile, b = b0 + bl;
        if (b >= O.B) continue;
        const uint4 x = philox4x32_10(make_uint4((uint32_t)g, (uint32_t)b, t, O.problem_id), k0, k1);
        double zz[4];
        box_muller(x.x, x.y, zz[0], zz[1]);
        box_muller(x.z, x.w, zz[2], zz[3]);
#pragma unroll
        for (int h = 0; h < 4; ++h)
            if (4 * g + h < D) z[bl][4 * g + h] = zz[h];
    }
    for (int e = threadIdx.x; e < D; e += blockDim.x) wofs[e] = (e / O.n_act) * n + O.act[e % O.n_act];
    __syncthreads();
    // lanes run over the tile's paths for one coordinate e: the row of L is
    // read once per coordinate (a broadcast) rather than once per lane
    for (int idx = threadIdx.x; idx < kSampleTile * D; idx += blockDim.x) {
        const int bl = idx % kSampleTile, e = idx / kSampleTile, b = b0 + bl;
        if (b >= O.B) continue;
        const double *Lr = O.L + (size_t)e * D;
        double s = O.mu[e];
        for (int e2 = 0; e2 <= e; ++e2) s = fma(Lr[e2], z[bl][e2], s);
        O.xi[(size_t)b * D + e] = s;
        O.W[(size_t)b * per + wofs[e]] = (float)s;
    }
    // joints that are not sampled take their hold value (one division per
    // waypoint entry, shared by the tile's paths)
    const int nb = min(kSampleTile, O.B - b0);
    for (int r = threadIdx.x; r < per; r += blockDim.x) {
        const JointDev J = P.joints[r % n];
        if (J.active) continue;
        for (int bl = 0; bl < nb; ++bl) O.W[(size_t)(b0 + bl) * per + r] = J.qhold;
    }
}

__global__ __launch_bounds__(256) void k_sample(PlanView P, OptView O) { sample_body(P, O, blockIdx.x); }

// batch: blockIdx.y = problem, blockIdx.x = tile of 16 paths
__global__ __launch_bounds__(256) void k_sample_batched(const BatchProblem *__restrict__ probs) {
    const BatchProblem &bp = probs[blockIdx.y];
    if ((int)blockIdx.x * kSampleTile >= bp.O.B) return;
    sample_body(bp.P, bp.O, blockIdx.x);
}

// ---------------------------------------------------------------------------
// selection: the nu smallest (cost, index) pairs, in rank order
// ---------------------------------------------------------------------------

constexpr int kSelThreads = 1024;
// populations up to this size, and those of up to kSelThreads that keep more
// than half of their paths, are ranked by counting (each thread compares its
// key with every other); the others take the radix select (measured: rank
// counting 21 us at B = 600, 32 us at B = 1024; radix 21 and 22 us, but 39 us
// at B = nu = 1024, where the elites' sort is the whole population's)
constexpr int kSelRankMax = 768;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *buf, uint32_t &total) {
    const int tid = threadIdx.x;
    buf[tid] = v;
    __syncthreads();
    for (int o = 1; o < kSelThreads; o <<= 1) {
        uint32_t a = tid >= o ? buf[tid - o] : 0u;
        __syncthreads();
        buf[tid] += a;
        __syncthreads();
    }
    total = buf[kSelThreads - 1];
    uint32_t incl = buf[tid];
    __syncthreads();
    return incl - v;
}

// LDS writes of this wave become visible to its other lanes
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ascending bitonic sort of np (a power of two, <= 4 * kSelThreads) 64-bit
// keys in LDS.  Wave w owns elements [256 w, 256 w + 256), four per lane, so
// the stages of stride below 256 touch one wave's elements only and need no
// workgroup barrier.  Ends with one.
__device__ __forceinline__ void bitonic_sort(uint64_t *a, int np) {
    const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const bool owner = w * 256 < np;
    bool wide_before = true;
    for (int size = 2; size <= np; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const bool wide = stride >= 256;
            if (wide || wide_before) __syncthreads();
            else wave_lds_sync();
            wide_before = wide;
            if (owner) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int i = w * 256 + k * 64 + lane, jx = i ^ stride;
                    if (i < np && jx > i) {
                        const bool up = (i & size) == 0;
                        const uint64_t x = a[i], y = a[jx];
                        if ((x > y) == up) { a[i] = y; a[jx] = x; }
                    }
                }
            }
        }
    }
    __syncthreads();
}

// the digit of a radix-select pass: the first bin where the running count
// reaches `remaining`, and how many of that bin are still to be taken (four
// bins per lane of wave 0, an inclusive scan of the lane sums)
__device__ __forceinline__ void select_digit(const uint32_t *hist, uint32_t remaining, uint32_t &s_digit,
                                             uint32_t &s_rem) {
    const int tid = threadIdx.x;
    if (tid < 64) {
        uint32_t h[4], sum = 0;
        for (int d = 0; d < 4; ++d) sum += h[d] = hist[4 * tid + d];
        uint32_t incl = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t up = __shfl_up(incl, o, 64);
            if (tid >= o) incl += up;
        }
        uint32_t cum = incl - sum;
        for (int d = 0; d < 4; ++d) {
            if (cum < remaining && cum + h[d] >= remaining) {
                s_digit = (uint32_t)(4 * tid + d);
                s_rem = remaining - cum;
            }
            cum += h[d];
        }
    }
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Radix select with PER keys per thread held in registers: slot j of thread
// t is path j kSelThreads + t.  Slots past B hold a key above every path's,
// and their indices lie above every path's, so they are never among the nu
// smallest (key, index) pairs and every slot can be processed alike.  Leaves
// the nu selected (relative key, index) pairs, unordered, in sorted[0, nu).
template <int PER>
__device__ __forceinline__ void select_regs(const float *__restrict__ cost, int B, int nu, uint32_t *hist,
                                            uint32_t *eqoff, uint64_t *sorted, uint32_t &s_digit, uint32_t &s_rem,
                                            uint32_t &s_count) {
    static_assert(PER % 8 == 0 && PER <= 64, "keys are loaded eight at a time; eqoff holds 64 slots");
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    // slot j reads cost[t + min(j kSelThreads, B - 1 - t)], always in bounds,
    // and keeps it when j kSelThreads <= B - 1 - t
    const float *ct = cost + tid;
    const int lim = B - 1 - tid;
    uint32_t key[PER];
#pragma unroll
    for (int j0 = 0; j0 < PER; j0 += 8) {
        float c[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) c[j] = ct[min((j0 + j) * kSelThreads, lim)];
#pragma unroll
        for (int j = 0; j < 8; ++j) key[j0 + j] = cost_key(c[j]);
    }
    // The keys are taken relative to the smallest one, and the digits run
    // over the bits of the span only: similar costs, whose keys share their
    // leading bytes, then spread over the first pass's bins instead of piling
    // onto a few (same-bin atomics serialise).  Slots past B get span + 1,
    // above every path's key; the order of the paths' keys is unchanged.
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        if (j * kSelThreads <= lim) {
            kmin = min(kmin, key[j]);
            kmax = max(kmax, key[j]);
        }
    }
    for (int o = 1; o < 64; o <<= 1) {
        kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, o, 64));
        kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, o, 64));
    }
    if (lane == 0) { hist[w] = kmin; hist[16 + w] = kmax; }
    __syncthreads();
    kmin = hist[0];
    kmax = hist[16];
    for (int x = 1; x < kSelThreads / 64; ++x) {
        kmin = min(kmin, hist[x]);
        kmax = max(kmax, hist[16 + x]);
    }
    __syncthreads();
    const uint32_t span1 = kmax - kmin + 1u;  // keys lie in [0x007FFFFF, 0xFF800000]: no wrap
    const int nb = 32 - __builtin_clz(span1);
#pragma unroll
    for (int j = 0; j < PER; ++j) key[j] = j * kSelThreads <= lim ? key[j] - kmin : span1;
    uint32_t prefix = 0, mask = 0, remaining = (uint32_t)nu;
    // most significant digit first (8 bits, the last one possibly fewer); a
    // wave whose counted keys share one digit adds them with one atomic
    for (int hi = nb; hi > 0;) {
        const int lo = hi > 8 ? hi - 8 : 0;
        const uint32_t dmask = (1u << (hi - lo)) - 1u;
        if (tid < 256) hist[tid] = 0;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const bool m = (key[j] & mask) == prefix;
            const uint64_t bm = __builtin_amdgcn_ballot_w64(m);
            if (bm) {
                const uint32_t d = (key[j] >> lo) & dmask;
                const int lead = __builtin_ctzll(bm);
                const uint32_t dl = (uint32_t)__builtin_amdgcn_readlane((int)d, lead);
                if (__builtin_amdgcn_ballot_w64(m && d == dl) == bm) {
                    if (lane == lead) atomicAdd(&hist[dl], (uint32_t)__builtin_popcountll(bm));
                } else if (m) {
                    atomicAdd(&hist[d], 1u);
                }
            }
        }
        __syncthreads();
        select_digit(hist, remaining, s_digit, s_rem);
        __syncthreads();
        prefix |= s_digit << lo;
        mask |= dmask << lo;
        remaining = s_rem;
        hi = lo;
    }
    // keys below the threshold, and the `remaining` lowest-index keys equal
    // to it: the equal keys are counted per (slot, wave), in index order, and
    // one wave turns the counts into offsets
    if (tid == 0) s_count = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint64_t be = __builtin_amdgcn_ballot_w64(key[j] == prefix);
        if (lane == 0) eqoff[j * 16 + w] = (uint32_t)__builtin_popcountll(be);
    }
    __syncthreads();
    if (tid < 64) {
        uint32_t c[16], sum = 0;
        for (int x = 0; x < 16; ++x) sum += c[x] = tid < PER ? eqoff[tid * 16 + x] : 0u;
        uint32_t incl = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t up = __shfl_up(incl, o, 64);
            if (tid >= o) incl += up;
        }
        uint32_t run = incl - sum;
        if (tid < PER)
            for (int x = 0; x < 16; ++x) { eqoff[tid * 16 + x] = run; run += c[x]; }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const bool eq = key[j] == prefix;
        const uint64_t be = __builtin_amdgcn_ballot_w64(eq);
        const bool take_eq = be && eq && eqoff[j * 16 + w] + lanes_below(be) < remaining;
        const bool sel = key[j] < prefix || take_eq;
        const uint64_t bm = __builtin_amdgcn_ballot_w64(sel);
        if (bm) {
            const int lead = __builtin_ctzll(bm);
            uint32_t base = 0;
            if (lane == lead) base = atomicAdd(&s_count, (uint32_t)__builtin_popcountll(bm));
            base = (uint32_t)__builtin_amdgcn_readlane((int)base, lead);
            if (sel) {
                // the key is copied to a fresh register first: a 64-bit store
                // straight from key[j] would make the register allocator keep
                // every key in the upper half of a register pair
                uint32_t kc;
                asm volatile("v_mov_b32 %0, %1" : "=v"(kc) : "v"(key[j]));
                sorted[base + lanes_below(bm)] = ((uint64_t)kc << 32) | (uint32_t)(j * kSelThreads + tid);
            }
        }
    }
}

__device__ __forceinline__ void select_body(const float *__restrict__ cost, int B, int nu,
                                            int32_t *__restrict__ elite) {
    __shared__ uint32_t hist[256];
    __shared__ uint32_t scanbuf[kSelThreads];
    __shared__ uint64_t sorted[CP_MAX_ELITES];
    __shared__ uint32_t s_digit, s_rem, s_count;
    const int tid = threadIdx.x;
    if (B <= kSelRankMax || (B <= kSelThreads && 2 * nu > B)) {
        // small populations: every path's rank in the (cost, index) order is
        // the number of smaller 64-bit keys, counted directly (broadcast LDS
        // reads); the first nu ranks are the elites
        if (tid < B) sorted[tid] = ((uint64_t)cost_key(cost[tid]) << 32) | (uint32_t)tid;
        __syncthreads();
        if (tid < B) {
            const uint64_t mine = sorted[tid];
            int rank = 0;
            for (int j = 0; j < B; ++j) rank += sorted[j] < mine ? 1 : 0;
            if (rank < nu) elite[rank] = tid;
        }
        return;
    }
    if (B <= 8 * kSelThreads) {
        select_regs<8>(cost, B, nu, hist, scanbuf, sorted, s_digit, s_rem, s_count);
    } else if (B <= 16 * kSelThreads) {
        select_regs<16>(cost, B, nu, hist, scanbuf, sorted, s_digit, s_rem, s_count);
    } else if (B <= 32 * kSelThreads) {
        select_regs<32>(cost, B, nu, hist, scanbuf, sorted, s_digit, s_rem, s_count);
    } else if (B <= 64 * kSelThreads) {
        select_regs<64>(cost, B, nu, hist, scanbuf, sorted, s_digit, s_rem, s_count);
    } else {
        // larger populations: the same radix select reading the costs from
        // global memory on every pass
        uint32_t prefix = 0, mask = 0, remaining = (uint32_t)nu;
        for (int pass = 0; pass < 4; ++pass) {
            const int shift = 24 - 8 * pass;
            if (tid < 256) hist[tid] = 0;
            __syncthreads();
            for (int i = tid; i < B; i += kSelThreads) {
                const uint32_t key = cost_key(cost[i]);
                if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
            }
            __syncthreads();
            select_digit(hist, remaining, s_digit, s_rem);
            __syncthreads();
            prefix |= s_digit << shift;
            mask |= 255u << shift;
            remaining = s_rem;
            __syncthreads();
        }
        // keys below the threshold, plus the `remaining` lowest-index keys
        // equal to it, from contiguous chunks in thread order
        const int chunk = (B + kSelThreads - 1) / kSelThreads;
        const int i0 = min(B, tid * chunk), i1 = min(B, i0 + chunk);
        uint32_t n_less = 0, n_eq = 0;
        for (int i = i0; i < i1; ++i) {
            const uint32_t key = cost_key(cost[i]);
            n_less += key < prefix;
            n_eq += key == prefix;
        }
        uint32_t tot;
        const uint32_t eq_before = block_exclusive_scan(n_eq, scanbuf, tot);
        const uint32_t take_eq = eq_before >= remaining ? 0u : min(n_eq, remaining - eq_before);
        const uint32_t off = block_exclusive_scan(n_less + take_eq, scanbuf, tot);
        uint32_t pos = off, eq_seen = 0;
        for (int i = i0; i < i1; ++i) {
            const uint32_t key = cost_key(cost[i]);
            bool sel = key < prefix;
            if (key == prefix) { sel = eq_seen < take_eq; ++eq_seen; }
            if (sel) sorted[pos++] = ((uint64_t)key << 32) | (uint32_t)i;
        }
    }
    int np = 1;
    while (np < nu) np <<= 1;
    for (int i = nu + tid; i < np; i += kSelThreads) sorted[i] = ~0ull;
    bitonic_sort(sorted, np);
    for (int r = tid; r < nu; r += kSelThreads) elite[r] = (int32_t)(uint32_t)(sorted[r] & 0xFFFFFFFFu);
}

__global__ __launch_bounds__(kSelThreads) void k_select(const float *__restrict__ cost, int B, int nu,
                                                        int32_t *__restrict__ elite) {
    select_body(cost, B, nu, elite);
}

// populations up to kSelThreads: the evaluation's per-path sums and the
// selection in one workgroup (each thread sums its own path, then ranks it)
__global__ __launch_bounds__(kSelThreads) void k_reduce_select(const double2 *__restrict__ partial, int slots, int ns,
                                                               float margin, float *__restrict__ cost,
                                                               float *__restrict__ min_dist, int B, int nu,
                                                               int32_t *__restrict__ elite) {
    if ((int)threadIdx.x < B) reduce_one(partial, slots, ns, margin, cost, min_dist, nullptr, threadIdx.x);
    __syncthreads();  // the radix select reads other threads' sums
    select_body(cost, B, nu, elite);
}

// batch: one workgroup per problem
__global__ __launch_bounds__(kSelThreads) void k_select_batched(const BatchProblem *__restrict__ probs) {
    const OptView &O = probs[blockIdx.x].O;
    select_body(O.cost, O.B, O.nu, O.elite0);
}

// ---------------------------------------------------------------------------
// gradient polish of the elites
// ---------------------------------------------------------------------------

__global__ void k_polish_gather(PlanView P, OptView O, float *__restrict__ dst) {
    const int per = P.K * P.n_joints;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < O.npol * per; idx += gridDim.x * blockDim.x) {
        const int i = idx / per, r = idx % per;
        dst[idx] = O.W[(size_t)O.elite0[i] * per + r];
    }
}

// elites re-ranked after polish: polished slots (index B + i) carry their new
// cost, the rest keep theirs; ties keep the earlier rank
__global__ __launch_bounds__(kSelThreads) void k_rerank(OptView O) {
    __shared__ uint64_t keys[CP_MAX_ELITES];
    const int nu = O.nu;
    int np = 1;
    while (np < nu) np <<= 1;
    for (int r = threadIdx.x; r < np; r += kSelThreads) {
        if (r < nu) {
            const float c = r < O.npol ? O.cost_p[r] : O.cost[O.elite0[r]];
            keys[r] = ((uint64_t)cost_key(c) << 32) | (uint32_t)r;
        } else {
            keys[r] = ~0ull;
        }
    }
    __syncthreads();
    bitonic_sort(keys, np);
    for (int r = threadIdx.x; r < nu; r += kSelThreads) {
        const int src = (int)(keys[r] & 0xFFFFFFFFu);
        O.elite[r] = src < O.npol ? O.B + src : O.elite0[src];
    }
}

// ---------------------------------------------------------------------------
// mean and covariance update (steps 4-6) and best-so-far
// ---------------------------------------------------------------------------

// One workgroup per 8 x 8 tile of the lower triangle of C, sixteen threads per
// entry.  Every workgroup first forms the means of its tile's rows and columns
// (the same arithmetic in every workgroup, so all hold identical values;
// diagonal tiles store theirs), then accumulates its entries about those
// means.  Elites are staged through LDS 256 at a time.
constexpr int kUpdTile = 8;
constexpr int kUpdParts = 16;  // interleaved partial sums per entry (elites j = part mod 16)
constexpr int kUpdThreads = kUpdTile * kUpdTile * kUpdParts;
constexpr int kUpdChunk = 256;
constexpr int kUpdTilesPerDim = (CP_MAX_DIM + kUpdTile - 1) / kUpdTile;
constexpr int kUpdTiles = kUpdTilesPerDim * (kUpdTilesPerDim + 1) / 2;

__device__ __forceinline__ double elite_value(const PlanView &P, const OptView &O, int idx, int e) {
    if (idx < O.B) return O.xi[(size_t)idx * O.D + e];
    const int k = e / O.n_act, a = e % O.n_act;
    return (double)O.Wp[((size_t)(idx - O.B) * P.K + k) * P.n_joints + O.act[a]];
}

__device__ __forceinline__ const float *elite_waypoints(const PlanView &P, const OptView &O, int idx) {
    const size_t per = (size_t)P.K * P.n_joints;
    return idx < O.B ? O.W + (size_t)idx * per : O.Wp + (size_t)(idx - O.B) * per;
}

__device__ __forceinline__ float elite_cost(const OptView &O, int idx) {
    return idx < O.B ? O.cost[idx] : O.cost_p[idx - O.B];
}

__device__ __forceinline__ void update_tile(const PlanView &P, const OptView &O, int t) {
    const int D = O.D, nu = O.nu, tid = threadIdx.x;
    const int nt = (D + kUpdTile - 1) / kUpdTile;
    int ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    const int tj = t - ti * (ti + 1) / 2;
    if (ti >= nt) return;  // whole workgroup
    const int r0 = ti * kUpdTile, c0 = tj * kUpdTile;
    const int part = tid / (kUpdTile * kUpdTile), ent = tid % (kUpdTile * kUpdTile);
    const int r = ent / kUpdTile, c = ent % kUpdTile;
    __shared__ double xr[kUpdChunk][kUpdTile], xc[kUpdChunk][kUpdTile];
    __shared__ double wch[kUpdChunk];
    __shared__ int ech[kUpdChunk];
    __shared__ double mr[kUpdTile], mc[kUpdTile];
    __shared__ double pm[kUpdParts][2 * kUpdTile], pc[kUpdParts][kUpdTile * kUpdTile];
    __shared__ int s_improved;
    // stage elites j0 .. j0 + nj - 1 of the tile's rows and columns (minus the
    // means once they are known)
    auto stage = [&](int j0, int nj, bool centred) {
        for (int i = tid; i < nj; i += kUpdThreads) {
            ech[i] = O.elite[j0 + i];
            wch[i] = O.w[j0 + i];
        }
        __syncthreads();
        if (O.npol == 0) {
            // every elite is a sample: each thread's loads are issued
            // together, at clamped (always valid) addresses
            constexpr int kPer = kUpdChunk * 2 * kUpdTile / kUpdThreads;
            static_assert(kPer * kUpdThreads == kUpdChunk * 2 * kUpdTile, "stage split");
            const int nslot = nj * 2 * kUpdTile;
            double v[kPer];
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                if (u * kUpdThreads >= nslot) break;
                const int idx = tid + u * kUpdThreads;
                const int jj = idx / (2 * kUpdTile), q = idx % (2 * kUpdTile);
                const int e = q < kUpdTile ? r0 + q : c0 + q - kUpdTile;
                v[u] = O.xi[(size_t)ech[min(jj, nj - 1)] * D + min(e, D - 1)];
            }
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                if (u * kUpdThreads >= nslot) break;
                const int idx = tid + u * kUpdThreads;
                const int jj = idx / (2 * kUpdTile), q = idx % (2 * kUpdTile);
                if (jj >= nj) continue;
                const bool row = q < kUpdTile;
                const int qq = row ? q : q - kUpdTile;
                const int e = (row ? r0 : c0) + qq;
                double x = e < D ? v[u] : 0.0;
                if (centred) x -= row ? mr[qq] : mc[qq];
                if (row) xr[jj][qq] = x;
                else xc[jj][qq] = x;
            }
        } else {
            for (int idx = tid; idx < nj * 2 * kUpdTile; idx += kUpdThreads) {
                const int jj = idx / (2 * kUpdTile), q = idx % (2 * kUpdTile);
                const bool row = q < kUpdTile;
                const int qq = row ? q : q - kUpdTile;
                const int e = (row ? r0 : c0) + qq;
                double x = e < D ? elite_value(P, O, ech[jj], e) : 0.0;
                if (centred) x -= row ? mr[qq] : mc[qq];
                if (row) xr[jj][qq] = x;
                else xc[jj][qq] = x;
            }
        }
        __syncthreads();
    };
    // Every sum over the elites is taken as 16 interleaved partial sums
    // (ranks j = part mod 16, each in rank order) added in part order: the
    // same arithmetic in every workgroup, whatever the launch.
    // means: sum_j w_j x_(j)
    double m = 0.0;
    for (int j0 = 0; j0 < nu; j0 += kUpdChunk) {
        const int nj = min(kUpdChunk, nu - j0);
        stage(j0, nj, false);
        if (ent < 2 * kUpdTile) {
            for (int jj = part; jj < nj; jj += kUpdParts)
                m = fma(wch[jj], ent < kUpdTile ? xr[jj][ent] : xc[jj][ent - kUpdTile], m);
        }
        __syncthreads();
    }
    if (ent < 2 * kUpdTile) pm[part][ent] = m;
    __syncthreads();
    if (tid < 2 * kUpdTile) {
        double s = pm[0][tid];
        for (int q = 1; q < kUpdParts; ++q) s += pm[q][tid];
        if (tid < kUpdTile) mr[tid] = s;
        else mc[tid - kUpdTile] = s;
    }
    __syncthreads();
    if (ti == tj && tid < kUpdTile && r0 + tid < D) O.mu[r0 + tid] = mr[tid];
    // covariance about the new mean: sum_j w_j (x_(j) - mu)(x_(j) - mu)^T + eps I
    const int e1 = r0 + r, e2 = c0 + c;
    const bool mine = e1 < D && e2 < D && e2 <= e1;
    double acc = 0.0;
    for (int j0 = 0; j0 < nu; j0 += kUpdChunk) {
        const int nj = min(kUpdChunk, nu - j0);
        stage(j0, nj, true);
        if (mine)
            for (int jj = part; jj < nj; jj += kUpdParts) acc = fma(wch[jj] * xr[jj][r], xc[jj][c], acc);
        __syncthreads();
    }
    pc[part][ent] = acc;
    __syncthreads();
    if (part == 0 && mine) {
        double v = pc[0][ent];
        for (int q = 1; q < kUpdParts; ++q) v += pc[q][ent];
        v += e1 == e2 ? O.eps : 0.0;
        O.C[(size_t)e1 * D + e2] = v;
        O.C[(size_t)e2 * D + e1] = v;
    }
    if (t != 0) return;
    // best-so-far: the iteration's best sample, then the best polished elite
    if (tid == 0) {
        int imp = -1;
        float bc = *O.best_cost;
        const float cb = O.cost[O.elite0[0]];
        if (cb < bc) { bc = cb; imp = O.elite0[0]; }
        if (O.npol > 0) {
            const float c1 = elite_cost(O, O.elite[0]);
            if (c1 < bc) { bc = c1; imp = O.elite[0]; }
        }
        if (imp >= 0) *O.best_cost = bc;
        s_improved = imp;
        *O.t = *O.t + 1;
    }
    __syncthreads();
    if (s_improved >= 0) {
        const float *src = elite_waypoints(P, O, s_improved);
        for (int i = tid; i < P.K * P.n_joints; i += kUpdThreads) O.best_W[i] = src[i];
    }
}

__global__ __launch_bounds__(kUpdThreads) void k_update(PlanView P, OptView O) { update_tile(P, O, blockIdx.x); }

__global__ __launch_bounds__(kUpdThreads) void k_update_batched(const BatchProblem *__restrict__ probs) {
    const BatchProblem &bp = probs[blockIdx.y];
    update_tile(bp.P, bp.O, blockIdx.x);
}

// ---------------------------------------------------------------------------
// lower Cholesky factor of C (double, in shared memory, packed lower
// triangle); if a pivot is not positive, retry with C + 10^k eps I, k = 1..3
// ---------------------------------------------------------------------------

constexpr int kCholThreads = 256;

__device__ __forceinline__ void chol_body(const OptView &O) {
    __shared__ double A[CP_MAX_DIM * (CP_MAX_DIM + 1) / 2];
    __shared__ double dg[CP_MAX_DIM];
    __shared__ int s_fail;
    const int D = O.D, tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6, nw = kCholThreads / 64;
    auto at = [](int i, int j) { return i * (i + 1) / 2 + j; };
    // Right-looking factorisation with one barrier per column: the phase that
    // applies column k to the trailing triangle also completes column k + 1
    // (its pivot, square root and division), since those entries receive
    // their last update in that phase.  Each entry keeps the order of its
    // updates, k ascending.  Pivots go to dg[], so no entry is read and
    // written by different threads within a phase.  A failed pivot (taken as
    // 1 to keep the arithmetic finite) is acted on once the attempt ends, so
    // every thread passes the same barriers.
    bool ok = false;
    for (int attempt = 0; attempt < 4 && !ok; ++attempt) {
        const double jitter = attempt == 0 ? 0.0 : O.eps * (attempt == 1 ? 10.0 : attempt == 2 ? 100.0 : 1000.0);
        for (int idx = tid; idx < D * D; idx += kCholThreads) {
            const int i = idx / D, j = idx % D;
            if (j <= i) A[at(i, j)] = O.C[idx] + (i == j ? jitter : 0.0);
        }
        if (tid == 0) s_fail = 0;
        __syncthreads();
        {
            const double piv = A[0];
            const double d = sqrt(piv > 0.0 ? piv : 1.0);
            if (tid == 0) {
                dg[0] = d;
                if (!(piv > 0.0)) s_fail = 1;
            }
            for (int i = 1 + tid; i < D; i += kCholThreads) A[at(i, 0)] /= d;
        }
        __syncthreads();
        for (int k = 0; k + 1 < D; ++k) {
            const int c = k + 1, m = D - c;
            // pivot of column c from its last update; every thread forms it
            const double lck = A[at(c, k)];
            const double piv = __builtin_fma(-lck, lck, A[at(c, c)]);
            const double d = sqrt(piv > 0.0 ? piv : 1.0);
            if (tid == 0) {
                dg[c] = d;
                if (!(piv > 0.0)) s_fail = 1;
            }
            // the trailing triangle rows c..D-1, columns c..i, flattened
            // row by row and dealt to threads four entries at a time; all
            // loads of a batch precede its stores
            const int T = m * (m + 1) / 2;
            for (int e0 = tid; e0 < T; e0 += 4 * kCholThreads) {
                double a[4], li[4], lj[4];
                int pos[4];
                bool col[4], act[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + u * kCholThreads;
                    act[u] = e > 0 && e < T;  // e == 0 is the pivot itself
                    if (!act[u]) continue;
                    int r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
                    if (r * (r + 1) / 2 > e) --r;
                    if ((r + 1) * (r + 2) / 2 <= e) ++r;
                    const int i = c + r, j = c + (e - r * (r + 1) / 2);
                    li[u] = A[at(i, k)];
                    lj[u] = A[at(j, k)];
                    pos[u] = at(i, j);
                    a[u] = A[pos[u]];
                    col[u] = j == c;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (!act[u]) continue;
                    const double v = __builtin_fma(-li[u], lj[u], a[u]);
                    A[pos[u]] = col[u] ? v / d : v;
                }
            }
            __syncthreads();
        }
        ok = !s_fail;
        __syncthreads();
    }
    if (!ok) {
        if (tid == 0) *O.status = 1;
        return;  // keep the previous factor
    }
    for (int idx = tid; idx < D * D; idx += kCholThreads) {
        const int i = idx / D, j = idx % D;
        O.L[idx] = j < i ? A[at(i, j)] : j == i ? dg[i] : 0.0;
    }
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// The same factorisation for D <= DM <= 64 in one wave and its registers:
// lane i holds row i, padded to DM with identity rows (the factor of
// diag(C, I) is diag(L, I)); column k's entries l_jk reach the other lanes
// by v_readlane into scalar registers.  Every entry receives the same
// operations in the same order as in chol_body (updates k ascending as
// fused multiply-adds, then the division by its column's pivot root), so the
// two give identical factors.
template <int DM>
__device__ __forceinline__ void chol_reg(const OptView &O) {
    const int D = O.D, lane = threadIdx.x & 63;
    double a[DM];
    double mydiag = 1.0;
    bool ok = false;
    for (int attempt = 0; attempt < 4 && !ok; ++attempt) {
        const double jitter = attempt == 0 ? 0.0 : O.eps * (attempt == 1 ? 10.0 : attempt == 2 ? 100.0 : 1000.0);
        // lower triangle of row `lane` (C is symmetric: column reads
        // coalesce); every lane loads an in-bounds entry unconditionally, so
        // all DM loads are in flight together
        const int lr = lane < D ? lane : D - 1;
        double cv[DM];
#pragma unroll
        for (int j = 0; j < DM; ++j) cv[j] = O.C[(size_t)(j < D ? j : D - 1) * D + lr];
#pragma unroll
        for (int j = 0; j < DM; ++j)
            a[j] = lane < D && j < D ? (j <= lane ? cv[j] + (j == lane ? jitter : 0.0) : 0.0) : (j == lane ? 1.0 : 0.0);
        bool fail = false;
#pragma unroll
        for (int k = 0; k < DM; ++k) {
            const double piv = readlane_f64(a[k], k);
            fail = fail || !(piv > 0.0);
            const double d = sqrt(piv > 0.0 ? piv : 1.0);
            if (lane == k) mydiag = d;
            a[k] = a[k] / d;
#pragma unroll
            for (int j = k + 1; j < DM; ++j) a[j] = __builtin_fma(-a[k], readlane_f64(a[k], j), a[j]);
        }
        ok = !fail;
    }
    if (!ok) {
        if (lane == 0) *O.status = 1;
        return;  // keep the previous factor
    }
    if (lane < D) {
#pragma unroll
        for (int j = 0; j < DM; ++j)
            if (j < D) O.L[(size_t)lane * D + j] = j < lane ? a[j] : j == lane ? mydiag : 0.0;
    }
}

// one workgroup per factorisation; D <= 32 and D <= 64 in the first wave's
// registers, larger D in shared memory
__device__ __forceinline__ void chol_any(const OptView &O) {
    if (O.D <= 64) {
        if (threadIdx.x >= 64) return;
        if (O.D <= 32)
            chol_reg<32>(O);
        else
            chol_reg<64>(O);
        return;
    }
    chol_body(O);
}

__global__ __launch_bounds__(kCholThreads) void k_chol(OptView O) { chol_any(O); }

__global__ __launch_bounds__(kCholThreads) void k_chol_batched(const BatchProblem *__restrict__ probs) {
    chol_any(probs[blockIdx.x].O);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_init_state(const PlanView &P, const OptView &O, float sigma0, hipStream_t st) {
    const int n = O.D * O.D;
    hipLaunchKernelGGL(k_init_state, dim3((n + 255) / 256), dim3(256), 0, st, P, O, sigma0);
    return hipGetLastError();
}

hipError_t launch_sample(const PlanView &P, const OptView &O, hipStream_t st) {
    hipLaunchKernelGGL(k_sample, dim3((O.B + kSampleTile - 1) / kSampleTile), dim3(256), 0, st, P, O);
    return hipGetLastError();
}

bool reduce_select_fits(int B) { return B <= kSelThreads; }

hipError_t launch_reduce_select(const double2 *partial, int slots, int ns, float margin, const OptView &O,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_select, dim3(1), dim3(kSelThreads), 0, st, partial, slots, ns, margin, O.cost,
                       O.min_dist, O.B, O.nu, O.elite0);
    return hipGetLastError();
}

hipError_t launch_select(const OptView &O, hipStream_t st) {
    hipLaunchKernelGGL(k_select, dim3(1), dim3(kSelThreads), 0, st, O.cost, O.B, O.nu, O.elite0);
    return hipGetLastError();
}

hipError_t launch_polish_gather(const PlanView &P, const OptView &O, float *dst, hipStream_t st) {
    const int n = O.npol * P.K * P.n_joints;
    hipLaunchKernelGGL(k_polish_gather, dim3((n + 255) / 256), dim3(256), 0, st, P, O, dst);
    return hipGetLastError();
}

hipError_t launch_rerank(const OptView &O, hipStream_t st) {
    hipLaunchKernelGGL(k_rerank, dim3(1), dim3(kSelThreads), 0, st, O);
    return hipGetLastError();
}

hipError_t launch_update(const PlanView &P, const OptView &O, hipStream_t st) {
    hipLaunchKernelGGL(k_update, dim3(kUpdTiles), dim3(kUpdThreads), 0, st, P, O);
    return hipGetLastError();
}

hipError_t launch_chol(const OptView &O, hipStream_t st) {
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(kCholThreads), 0, st, O);
    return hipGetLastError();
}

hipError_t launch_batch_sample(const BatchProblem *probs, int n, int max_B, hipStream_t st) {
    hipLaunchKernelGGL(k_sample_batched, dim3((max_B + kSampleTile - 1) / kSampleTile, n), dim3(256), 0, st, probs);
    return hipGetLastError();
}

hipError_t launch_batch_iteration(const BatchProblem *probs, double2 *partial, int n, int max_B, const int2 *items,
                                  int n_items, int rounds, int grid, bool cull, hipStream_t st) {
    hipError_t e = launch_batch_sample(probs, n, max_B, st);
    if (e != hipSuccess) return e;
    if ((e = launch_batch_eval(probs, partial, n, max_B, items, n_items, rounds, grid, cull, st)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_select_batched, dim3(n), dim3(kSelThreads), 0, st, probs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_update_batched, dim3(kUpdTiles, n), dim3(kUpdThreads), 0, st, probs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_chol_batched, dim3(n), dim3(kCholThreads), 0, st, probs);
    return hipGetLastError();
}

}  // namespace cp
