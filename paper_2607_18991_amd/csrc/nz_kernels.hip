// nz_kernels.hip -- CDNA4 (gfx950) kernels of the Newman-Ziff first-spanning
// sweep on sc(5) (Malarz & Woloszyn, Sec. II.B; neighbourhoods of Sec. II.A.2).
//
// Pipeline per chunk of samples (all launched on one stream):
//   nz_clear_kernel    zero the bucket counters and per-sample state;
//   nz_keys_kernel     Philox4x32-10 key of every site (integer VALU bound);
//                      sites below the prefill threshold T0 are occupied at once
//                      (bitset word per 32 sites, parent = self, site list);
//                      sites in the key band [T0, T0 + nb << shift) are appended
//                      to the bucket of their key;
//   nz_hook/compress/  bulk connected components of the prefilled sites
//   accum kernels      (hook-and-compress with CAS links, then cluster sizes and
//                      border flags into the root word); a state that already
//                      spans is flagged for backoff;
//   nz_sort_kernel     each bucket sorted by (key, site) in LDS (bitonic);
//                      concatenated buckets are exactly the occupation order;
//   nz_sweep_kernel    persistent: every wave pops a sample (longest first) and
//                      adds its band sites one at a time; the z neighbour checks
//                      of a site are spread over the 64 lanes, occupied
//                      neighbours find their roots in parallel, the largest
//                      cluster absorbs the others, and the root word's two border
//                      flags decide spanning.
#include <hip/hip_runtime.h>

#include "nz_internal.h"

namespace nz {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): per round, counter words
// 0 and 2 are multiplied by two fixed odd constants; the high halves, xor-ed
// with words 1/3 and the round key, and the low halves form the next counter.
// The key advances by the Weyl increments between rounds.

constexpr uint32_t kPhiloxMulA = 0xD2511F53u;
constexpr uint32_t kPhiloxMulB = 0xCD9E8D57u;
constexpr uint32_t kWeylA = 0x9E3779B9u;
constexpr uint32_t kWeylB = 0xBB67AE85u;

__device__ __forceinline__ uint64_t site_key(uint32_t seed_lo, uint32_t seed_hi,
                                             uint32_t smp_lo, uint32_t smp_hi, uint32_t site)
{
    uint32_t c0 = site, c1 = smp_lo, c2 = smp_hi, c3 = 0u;  // word 3: domain tag 0
    uint32_t k0 = seed_lo, k1 = seed_hi;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a_hi = __umulhi(kPhiloxMulA, c0);
        const uint32_t a_lo = kPhiloxMulA * c0;
        const uint32_t b_hi = __umulhi(kPhiloxMulB, c2);
        const uint32_t b_lo = kPhiloxMulB * c2;
        c0 = b_hi ^ c1 ^ k0;
        c1 = b_lo;
        c2 = a_hi ^ c3 ^ k1;
        c3 = a_lo;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return (static_cast<uint64_t>(c1) << 32) | c0;
}

// floor(n / L) for n < 2^32 with magic = ceil(2^64 / L) (0 for L = 1).
__device__ __forceinline__ uint32_t div_by_L(uint32_t n, uint64_t magic)
{
    return static_cast<uint32_t>(__umul64hi(static_cast<uint64_t>(n), magic));
}

// Packed coordinates x0 | x1 << 6 | ... | x4 << 24.  Packed values order like
// site indices (x4 most significant), so (key, packed) sorts like (key, site).
__device__ __forceinline__ uint32_t pack_coords(uint32_t i, uint32_t L, uint64_t magic)
{
    uint32_t pc = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t q = div_by_L(i, magic);
        pc |= (i - q * L) << (6 * j);
        i = q;
    }
    return pc | (i << 24);
}

// Bits (5j + d + 2) for the d in [-2, 2] that keep x + d inside [0, L).
__device__ __forceinline__ uint32_t allowed_axis(int32_t x, int32_t L)
{
    const int32_t lo = max(0, 2 - x);
    const int32_t hi = min(4, L + 1 - x);
    return hi >= lo ? ((2u << hi) - (1u << lo)) : 0u;
}

// Relaxed atomics: wavefront scope for state private to one wave, agent scope
// for state shared by all workgroups (bulk connected components).
template <typename T>
__device__ __forceinline__ T ld_w(T *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT); }
template <typename T>
__device__ __forceinline__ void st_w(T *p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT); }
template <typename T>
__device__ __forceinline__ T ld_a(T *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
template <typename T>
__device__ __forceinline__ void st_a(T *p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

template <typename T>
__device__ __forceinline__ T bcast(T v, int lane)
{
    return static_cast<T>(__builtin_amdgcn_readlane(static_cast<int>(v), lane));
}

// ---------------------------------------------------------------------------
// Clearing: bucket counters and per-sample state of a chunk.

__global__ __launch_bounds__(256) void nz_clear_kernel(const NzSample *__restrict__ desc, const int32_t *__restrict__ list,
                                                       int32_t nsamp, uint8_t *__restrict__ ws, NzState *__restrict__ state)
{
    if (static_cast<int32_t>(blockIdx.x) >= nsamp) return;
    const int sid = list ? list[blockIdx.x] : static_cast<int>(blockIdx.x);
    const NzSample &d = desc[sid];
    uint32_t *counts = reinterpret_cast<uint32_t *>(ws + d.off_counts);
    for (int b = threadIdx.x; b < d.nb; b += blockDim.x) counts[b] = 0u;
    if (threadIdx.x == 0) {
        NzState s;
        s.status = NZ_ST_PENDING;
        s.nstar = 0;
        s.mass = 0;
        s.n0 = 0;
        state[sid] = s;
    }
}

// ---------------------------------------------------------------------------
// Keys, prefill occupancy and band bucketing.  A block covers
// KEYS_THREADS * KEYS_ITERS consecutive sites of one sample; each wave handles
// 64 consecutive sites per iteration so that a ballot yields two bitset words.

constexpr int KEYS_THREADS = 256;
constexpr int KEYS_ITERS = 16;
constexpr int KEYS_SITES_PER_BLOCK = KEYS_THREADS * KEYS_ITERS;

__global__ __launch_bounds__(KEYS_THREADS) void nz_keys_kernel(const NzSample *__restrict__ desc,
                                                               const int32_t *__restrict__ list, int32_t first,
                                                               int32_t blocks_per_sample, uint8_t *__restrict__ ws,
                                                               NzState *__restrict__ state)
{
    // prefilled sites of this block, staged in LDS and appended to the
    // sample's list with one global atomic per block
    __shared__ uint32_t pre_sites[KEYS_SITES_PER_BLOCK];
    __shared__ uint32_t pre_count, pre_base;
    const int which = static_cast<int>(blockIdx.x) / blocks_per_sample;
    const int sid = list ? list[first + which] : first + which;
    const int blk = static_cast<int>(blockIdx.x) % blocks_per_sample;
    const NzSample &d = desc[sid];
    const uint32_t N = static_cast<uint32_t>(d.N);
    const uint32_t L = static_cast<uint32_t>(d.L);
    const uint64_t magic = d.magic;
    const uint64_t T0 = d.T0;
    const int32_t shift = d.shift;
    const uint64_t nb = static_cast<uint64_t>(d.nb);
    const uint32_t cap = static_cast<uint32_t>(d.cap);
    const uint32_t seed_lo = static_cast<uint32_t>(d.seed), seed_hi = static_cast<uint32_t>(d.seed >> 32);
    const uint32_t smp_lo = static_cast<uint32_t>(d.sample), smp_hi = static_cast<uint32_t>(d.sample >> 32);

    uint32_t *occ = reinterpret_cast<uint32_t *>(ws + d.off_occ);
    int32_t *par = reinterpret_cast<int32_t *>(ws + d.off_par);
    uint64_t *keys = reinterpret_cast<uint64_t *>(ws + d.off_keys);
    uint32_t *sites = reinterpret_cast<uint32_t *>(ws + d.off_sites);
    uint32_t *counts = reinterpret_cast<uint32_t *>(ws + d.off_counts);
    uint32_t *prefix = reinterpret_cast<uint32_t *>(ws + d.off_prefix);

    const uint32_t lane = lane_id();
    const uint32_t block_base = static_cast<uint32_t>(blk) * KEYS_SITES_PER_BLOCK;
    if (threadIdx.x == 0) pre_count = 0u;
    __syncthreads();
    for (int it = 0; it < KEYS_ITERS; ++it) {
        const uint32_t wbase = block_base + it * KEYS_THREADS + (threadIdx.x & ~63u);
        if (wbase >= N) break;
        const uint32_t i = wbase + lane;
        const bool valid = i < N;
        const uint64_t K = site_key(seed_lo, seed_hi, smp_lo, smp_hi, i);
        const bool pre = valid && K < T0;
        const uint64_t bal = __ballot(pre);
        // Every lane stores: even lanes the low word, odd lanes the high word of
        // the ballot (identical values per address).  No lane-conditional block
        // sits next to a cross-lane operation inside this loop.  The bitset is
        // padded to whole 64-site words, so both words exist.
        occ[(wbase >> 5) + (lane & 1u)] = static_cast<uint32_t>(bal >> (32u * (lane & 1u)));
        if (pre) {
            par[i] = static_cast<int32_t>(i);
            pre_sites[atomicAdd(&pre_count, 1u)] = i;
        }
        if (valid && !pre) {
            const uint64_t b = (K - T0) >> shift;
            if (b < nb) {
                const uint32_t slot = atomicAdd(&counts[b], 1u);
                if (slot < cap) {
                    keys[b * cap + slot] = K;
                    sites[b * cap + slot] = pack_coords(i, L, magic);
                }
            }
        }
    }
    __syncthreads();
    const uint32_t cnt = pre_count;
    if (cnt) {
        if (threadIdx.x == 0) pre_base = atomicAdd(reinterpret_cast<uint32_t *>(&state[sid].n0), cnt);
        __syncthreads();
        const uint32_t base = pre_base;
        for (uint32_t k = threadIdx.x; k < cnt; k += KEYS_THREADS) {
            const uint32_t pos = base + k;
            if (pos < static_cast<uint32_t>(d.prefix_cap)) prefix[pos] = pre_sites[k];
        }
    }
}

// ---------------------------------------------------------------------------
// Bucket sort: one workgroup per (sample, bucket); bitonic network in LDS over
// (key, packed site) pairs padded to a power of two; sorted packed sites are
// written back in place.  Over-full buckets are left alone (the sweep reports
// them if it reaches one).

constexpr int SORT_THREADS = 256;

__device__ __forceinline__ bool pair_greater(uint64_t ka, uint32_t pa, uint64_t kb, uint32_t pb)
{
    return ka > kb || (ka == kb && pa > pb);
}

__global__ __launch_bounds__(SORT_THREADS) void nz_sort_kernel(const NzSample *__restrict__ desc, int32_t nsamp,
                                                               int32_t max_nb, uint8_t *__restrict__ ws)
{
    extern __shared__ uint64_t sort_lds[];
    const int64_t items = static_cast<int64_t>(nsamp) * max_nb;
    for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {
        const int sid = static_cast<int>(item / max_nb);
        const int b = static_cast<int>(item % max_nb);
        const NzSample &d = desc[sid];
        if (b >= d.nb) continue;
        const uint32_t *counts = reinterpret_cast<const uint32_t *>(ws + d.off_counts);
        const uint32_t cnt = counts[b];
        const uint32_t cap = static_cast<uint32_t>(d.cap);
        if (cnt <= 1u || cnt > cap) continue;
        uint32_t P = 1;
        while (P < cnt) P <<= 1;
        uint64_t *k = sort_lds;
        uint32_t *p = reinterpret_cast<uint32_t *>(sort_lds + P);
        const uint64_t *gk = reinterpret_cast<const uint64_t *>(ws + d.off_keys) + static_cast<uint64_t>(b) * cap;
        uint32_t *gp = reinterpret_cast<uint32_t *>(ws + d.off_sites) + static_cast<uint64_t>(b) * cap;
        for (uint32_t i = threadIdx.x; i < P; i += SORT_THREADS) {
            if (i < cnt) {
                k[i] = gk[i];
                p[i] = gp[i];
            } else {
                k[i] = ~0ull;
                p[i] = ~0u;
            }
        }
        __syncthreads();
        for (uint32_t size = 2; size <= P; size <<= 1) {
            for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                for (uint32_t i = threadIdx.x; i < P; i += SORT_THREADS) {
                    const uint32_t j = i ^ stride;
                    if (j > i) {
                        const bool up = (i & size) == 0;
                        const uint64_t ki = k[i], kj = k[j];
                        const uint32_t pi = p[i], pj = p[j];
                        if (pair_greater(ki, pi, kj, pj) == up) {
                            k[i] = kj; k[j] = ki;
                            p[i] = pj; p[j] = pi;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t i = threadIdx.x; i < cnt; i += SORT_THREADS) gp[i] = p[i];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Bulk connected components of the prefilled sites (hook and compress).
// During this phase par[i] is a plain parent index and a root points to
// itself; every access is an agent-scope atomic because all workgroups work on
// the same forest at once.  Links always go from the larger root index to the
// smaller, so a CAS that finds its root unchanged can never form a cycle.

__device__ __forceinline__ int32_t cc_find(int32_t *par, int32_t x)
{
    int32_t p = ld_a(&par[x]);
    while (p != x) {
        const int32_t g = ld_a(&par[p]);
        if (g != p) st_a(&par[x], g);   // halving: x skips to its grandparent
        x = p;
        p = g;
    }
    return x;
}

__global__ __launch_bounds__(256) void nz_hook_kernel(const NzSample *__restrict__ desc, const int32_t *__restrict__ list,
                                                      const NzOffset *__restrict__ tabs, uint8_t *__restrict__ ws,
                                                      NzState *__restrict__ state)
{
    const int sid = list[blockIdx.y];
    const NzSample &d = desc[sid];
    const int32_t n0 = state[sid].n0;
    if (n0 > d.prefix_cap) return;
    const int32_t L = d.L;
    const int32_t zh = d.z >> 1;        // the first half of a table holds one of each +-d pair
    const uint64_t magic = d.magic;
    int32_t *par = reinterpret_cast<int32_t *>(ws + d.off_par);
    const uint32_t *occ = reinterpret_cast<const uint32_t *>(ws + d.off_occ);
    const uint32_t *prefix = reinterpret_cast<const uint32_t *>(ws + d.off_prefix);
    const NzOffset *tab = tabs + d.tab;
    const int64_t items = static_cast<int64_t>(n0) * zh;
    for (int64_t it = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; it < items;
         it += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int32_t s = static_cast<int32_t>(prefix[it / zh]);
        const NzOffset o = tab[it % zh];
        const uint32_t pc = pack_coords(static_cast<uint32_t>(s), static_cast<uint32_t>(L), magic);
        const uint32_t A = allowed_axis(pc & 63, L) | (allowed_axis((pc >> 6) & 63, L) << 5) |
                           (allowed_axis((pc >> 12) & 63, L) << 10) | (allowed_axis((pc >> 18) & 63, L) << 15) |
                           (allowed_axis(pc >> 24, L) << 20);
        if (o.code & ~A) continue;
        const int32_t t = s + o.stride;
        if (!((occ[t >> 5] >> (t & 31)) & 1u)) continue;
        int32_t u = cc_find(par, s);
        int32_t v = cc_find(par, t);
        while (u != v) {
            if (u < v) { const int32_t w = u; u = v; v = w; }
            int32_t expected = u;
            if (__hip_atomic_compare_exchange_strong(&par[u], &expected, v, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT))
                break;
            u = cc_find(par, expected);
            v = cc_find(par, v);
        }
    }
}

__device__ __forceinline__ uint32_t border_flags(uint32_t s, uint32_t L, uint64_t magic)
{
    const uint32_t x0 = s - div_by_L(s, magic) * L;
    return (x0 == 0 ? NZ_FLO : 0u) | (x0 == L - 1 ? NZ_FHI : 0u);
}

// Compress: every member points straight at its root, and every root takes its
// root word (size 1 plus its own border flags).  Each thread writes only its
// own entry and walks the forest read-only: a halving write here could replace
// an entry another thread has already pointed at its root with a non-root
// ancestor.  Roots never change in this kernel, so a walk stops at an entry that
// points to itself or already holds a root word.
__global__ __launch_bounds__(256) void nz_compress_kernel(const NzSample *__restrict__ desc, const int32_t *__restrict__ list,
                                                          uint8_t *__restrict__ ws, NzState *__restrict__ state)
{
    const int sid = list[blockIdx.y];
    const NzSample &d = desc[sid];
    const int32_t n0 = state[sid].n0;
    if (n0 > d.prefix_cap) return;
    const uint32_t L = static_cast<uint32_t>(d.L);
    int32_t *par = reinterpret_cast<int32_t *>(ws + d.off_par);
    const uint32_t *prefix = reinterpret_cast<const uint32_t *>(ws + d.off_prefix);
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n0; k += gridDim.x * blockDim.x) {
        const int32_t s = static_cast<int32_t>(prefix[k]);
        int32_t r = s;
        int32_t p = ld_a(&par[r]);
        while (p >= 0 && p != r) {
            r = p;
            p = ld_a(&par[r]);
        }
        if (r == s) {
            const uint32_t fl = border_flags(static_cast<uint32_t>(s), L, d.magic);
            st_a(&par[s], static_cast<int32_t>(NZ_ROOT | fl | 1u));
            if (fl == NZ_FLAGS) state[sid].status = NZ_ST_BACKOFF;   // L = 1: one site spans
        } else {
            st_a(&par[s], r);
        }
    }
}

// Sizes and border flags of the prefilled clusters: members add themselves to
// their root word.  The flag OR returns the previous word, so the member that
// completes a root's pair of border flags sees it: the state already spans and
// the sample backs off.
__global__ __launch_bounds__(256) void nz_accum_kernel(const NzSample *__restrict__ desc, const int32_t *__restrict__ list,
                                                       uint8_t *__restrict__ ws, NzState *__restrict__ state)
{
    const int sid = list[blockIdx.y];
    const NzSample &d = desc[sid];
    const int32_t n0 = state[sid].n0;
    if (n0 > d.prefix_cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) state[sid].status = NZ_ST_PREFIX;
        return;
    }
    const uint32_t L = static_cast<uint32_t>(d.L);
    int32_t *par = reinterpret_cast<int32_t *>(ws + d.off_par);
    const uint32_t *prefix = reinterpret_cast<const uint32_t *>(ws + d.off_prefix);
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n0; k += gridDim.x * blockDim.x) {
        const int32_t s = static_cast<int32_t>(prefix[k]);
        const int32_t r = par[s];
        if (r >= 0) {
            uint32_t *root = reinterpret_cast<uint32_t *>(&par[r]);
            atomicAdd(root, 1u);
            const uint32_t fl = border_flags(static_cast<uint32_t>(s), L, d.magic);
            if (fl) {
                const uint32_t old = atomicOr(root, fl);
                if (((old | fl) & NZ_FLAGS) == NZ_FLAGS) state[sid].status = NZ_ST_BACKOFF;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The sweep.  RES selects where the per-sample state of the running wave lives:
//   RES_HBM  bitset and parents in the workspace (HBM / L2);
//   RES_OCC  bitset in this wave's LDS slice, parents in HBM;
//   RES_ALL  bitset and parents in LDS.
// NCH = number of 64-offset chunks the kernel is compiled for (z <= 64 * NCH).

enum { RES_HBM = 0, RES_OCC = 1, RES_ALL = 2 };

template <int RES>
struct SweepMem {
    uint32_t *occ_g;
    int32_t *par_g;
    uint32_t lbase;     // first LDS word of this wave's slice
    uint32_t occ_words; // bitset words (padded to 64 sites)

    __device__ __forceinline__ uint32_t occ_ld(uint32_t *lds, uint32_t w) const
    {
        if constexpr (RES == RES_HBM) return ld_w(&occ_g[w]);
        else return ld_w(&lds[lbase + w]);
    }
    __device__ __forceinline__ void occ_st(uint32_t *lds, uint32_t w, uint32_t v) const
    {
        if constexpr (RES == RES_HBM) st_w(&occ_g[w], v);
        else st_w(&lds[lbase + w], v);
    }
    __device__ __forceinline__ int32_t par_ld(uint32_t *lds, int32_t i) const
    {
        if constexpr (RES == RES_ALL) return static_cast<int32_t>(ld_w(&lds[lbase + occ_words + i]));
        else return ld_w(&par_g[i]);
    }
    __device__ __forceinline__ void par_st(uint32_t *lds, int32_t i, int32_t v) const
    {
        if constexpr (RES == RES_ALL) st_w(&lds[lbase + occ_words + i], static_cast<uint32_t>(v));
        else st_w(&par_g[i], v);
    }
};

// Root of x with path halving; returns the root index and its root word.
template <int RES>
__device__ __forceinline__ void sweep_find(const SweepMem<RES> &m, uint32_t *lds, int32_t x, int32_t &root, uint32_t &word)
{
    int32_t v = m.par_ld(lds, x);
    while (v >= 0) {
        const int32_t g = m.par_ld(lds, v);
        if (g < 0) {
            x = v;
            v = g;
            break;
        }
        m.par_st(lds, x, g);
        x = g;
        v = m.par_ld(lds, x);
    }
    root = x;
    word = static_cast<uint32_t>(v);
}

// Merge the D distinct roots held by lanes 0..D-1 (lroot/lword) into the largest
// one (ties: smaller index).  Returns the surviving root; total size and flags
// through the references.
template <int RES>
__device__ __forceinline__ int32_t sweep_merge(const SweepMem<RES> &m, uint32_t *lds, int D, int32_t lroot, uint32_t lword,
                                               uint32_t &total, uint32_t &flags)
{
    const uint32_t lane = lane_id();
    int32_t best = bcast(lroot, 0);
    uint32_t bestsz = bcast(lword, 0) & NZ_SIZE;
    total = 0;
    flags = 0;
    for (int l = 0; l < D; ++l) {
        const int32_t r = bcast(lroot, l);
        const uint32_t w = bcast(lword, l);
        const uint32_t sz = w & NZ_SIZE;
        total += sz;
        flags |= w & NZ_FLAGS;
        if (sz > bestsz || (sz == bestsz && r < best)) {
            best = r;
            bestsz = sz;
        }
    }
    if (static_cast<int>(lane) < D && lroot != best) m.par_st(lds, lroot, best);
    // every lane stores the same root word (no lane-conditional block here)
    m.par_st(lds, best, static_cast<int32_t>(NZ_ROOT | flags | total));
    return best;
}

struct SweepOut {
    int32_t *nstar;
    int32_t *mass;
    const int32_t *out_index; // per sample: position in the caller's output arrays
};

template <int NCH, int RES>
__global__ void nz_sweep_kernel(NzSweepArgs a, SweepOut out)
{
    extern __shared__ uint32_t lds[];
    __shared__ int32_t claim[16];   // per-wave work claim
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x >> 6;

    for (;;) {
        // One lane claims the next queue entry and publishes it through LDS;
        // every lane then reads the slot, so no cross-lane read ever depends on
        // which lanes took a lane-conditional branch.
        if (lane == 0) claim[wave] = atomicAdd(a.qhead, 1);
        __builtin_amdgcn_wave_barrier();
        const int qi = __builtin_amdgcn_readfirstlane(ld_w(&claim[wave]));
        __builtin_amdgcn_wave_barrier();
        if (qi >= a.nqueue) break;
        const int sid = a.queue[qi];
        const int32_t status0 = a.state[sid].status;
        if (status0 != NZ_ST_PENDING) continue;
        const NzSample &d = a.desc[sid];
        const int32_t L = d.L;
        const int32_t N = d.N;
        const int32_t z = d.z;
        const int32_t nb = d.nb;
        const uint32_t cap = static_cast<uint32_t>(d.cap);
        const bool prefilled = d.T0 != 0;
        const int dcap = a.dcap;

        SweepMem<RES> m;
        m.occ_g = reinterpret_cast<uint32_t *>(a.ws + d.off_occ);
        m.par_g = reinterpret_cast<int32_t *>(a.ws + d.off_par);
        m.lbase = wave * a.lds_words;
        m.occ_words = static_cast<uint32_t>(((N + 63) >> 6) << 1);
        if constexpr (RES != RES_HBM) {
            for (uint32_t w = lane; w < m.occ_words; w += 64) lds[m.lbase + w] = prefilled ? m.occ_g[w] : 0u;
            if constexpr (RES == RES_ALL) {
                if (prefilled)
                    for (int32_t i = lane; i < N; i += 64) lds[m.lbase + m.occ_words + i] = static_cast<uint32_t>(m.par_g[i]);
            }
        } else if (!prefilled) {
            // the keys kernel wrote an all-zero bitset; nothing to do
        }

        const NzOffset *tab = a.tabs + d.tab;
        int32_t ostride[NCH];
        uint32_t ocode[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int32_t j = c * 64 + static_cast<int32_t>(lane);
            if (j < z) {
                const NzOffset o = tab[j];
                ostride[c] = o.stride;
                ocode[c] = o.code;
            } else {
                ostride[c] = 0;
                ocode[c] = 0xFFFFFFFFu;   // never inside: bits above 25 are never allowed
            }
        }

        const uint32_t *counts = reinterpret_cast<const uint32_t *>(a.ws + d.off_counts);
        const uint32_t *sites = reinterpret_cast<const uint32_t *>(a.ws + d.off_sites);
        int32_t r = a.state[sid].n0;   // sites already occupied
        int32_t status = NZ_ST_BAND;
        int32_t nstar = 0, mass = 0;

        for (int32_t b = 0; b < nb && status == NZ_ST_BAND; ++b) {
            const uint32_t cnt = counts[b];
            if (cnt > cap) {
                status = NZ_ST_BUCKET;
                break;
            }
            const uint32_t *bs = sites + static_cast<uint64_t>(b) * cap;
            for (uint32_t j0 = 0; j0 < cnt && status == NZ_ST_BAND; j0 += 64) {
                const uint32_t mine = (j0 + lane < cnt) ? bs[j0 + lane] : 0u;
                const uint32_t mcount = min(64u, cnt - j0);
                for (uint32_t jj = 0; jj < mcount; ++jj) {
                    const uint32_t pc = bcast(mine, static_cast<int>(jj));
                    const int32_t x0 = pc & 63, x1 = (pc >> 6) & 63, x2 = (pc >> 12) & 63, x3 = (pc >> 18) & 63,
                                  x4 = pc >> 24;
                    const int32_t s = x0 + L * (x1 + L * (x2 + L * (x3 + L * x4)));
                    const uint32_t A = allowed_axis(x0, L) | (allowed_axis(x1, L) << 5) | (allowed_axis(x2, L) << 10) |
                                       (allowed_axis(x3, L) << 15) | (allowed_axis(x4, L) << 20);
                    const uint32_t fl = (x0 == 0 ? NZ_FLO : 0u) | (x0 == L - 1 ? NZ_FHI : 0u);
                    ++r;

                    // neighbour occupancy: issue every chunk's load before using any
                    uint32_t word[NCH];
                    int32_t tn[NCH];
                    bool inb[NCH];
                    const uint32_t own = m.occ_ld(lds, static_cast<uint32_t>(s) >> 5);
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        inb[c] = (ocode[c] & ~A) == 0u;
                        tn[c] = s + ostride[c];
                        word[c] = inb[c] ? m.occ_ld(lds, static_cast<uint32_t>(tn[c]) >> 5) : 0u;
                    }
                    // all lanes store the same updated word of s (this wave is the
                    // only writer of the sample's bitset)
                    m.occ_st(lds, static_cast<uint32_t>(s) >> 5, own | (1u << (s & 31)));

                    // distinct roots: lanes 0..D-1 hold (root, root word); entry 0 is s itself
                    int32_t lroot = s;
                    uint32_t lword = NZ_ROOT | fl | 1u;
                    int D = 1;
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        const bool o = inb[c] && ((word[c] >> (tn[c] & 31)) & 1u);
                        uint64_t mk = __ballot(o);
                        if (!mk) continue;
                        int32_t root = 0;
                        uint32_t rw = 0;
                        if (o) sweep_find<RES>(m, lds, tn[c], root, rw);
                        bool stale = false;   // a flush since these finds may have linked their roots
                        while (mk) {
                            const int l = __builtin_ctzll(mk);
                            mk &= mk - 1;
                            int32_t rr = bcast(root, l);
                            uint32_t rrw = bcast(rw, l);
                            if (stale) sweep_find<RES>(m, lds, rr, rr, rrw);
                            if (__ballot(static_cast<int>(lane) < D && lroot == rr)) continue;
                            if (D == dcap) {
                                // list full: merge what we have and keep only the survivor;
                                // rr is not in the list, so the flush leaves it a root
                                uint32_t tot, flg;
                                const int32_t w = sweep_merge<RES>(m, lds, D, lroot, lword, tot, flg);
                                lroot = lane == 0 ? w : lroot;
                                lword = lane == 0 ? (NZ_ROOT | flg | tot) : lword;
                                D = 1;
                                stale = true;
                            }
                            lroot = static_cast<int>(lane) == D ? rr : lroot;
                            lword = static_cast<int>(lane) == D ? rrw : lword;
                            ++D;
                        }
                    }
                    uint32_t total, flags;
                    sweep_merge<RES>(m, lds, D, lroot, lword, total, flags);
                    if (flags == NZ_FLAGS) {
                        status = NZ_ST_DONE;
                        nstar = r;
                        mass = static_cast<int32_t>(total);
                        break;
                    }
                }
            }
        }
        if (status == NZ_ST_BAND && d.full) {
            status = NZ_ST_DONE;   // the whole lattice is occupied and never spans
            nstar = 0;
            mass = 0;
        }
        // every lane stores the same values
        a.state[sid].status = status;
        a.state[sid].nstar = nstar;
        a.state[sid].mass = mass;
        if (status == NZ_ST_DONE) {
            const int32_t o = out.out_index[sid];
            out.nstar[o] = nstar;
            if (out.mass) out.mass[o] = mass;
        }
    }
}

}  // namespace nz

// ---------------------------------------------------------------------------
// Host-side launchers (internal to the library).

#include "nz_launch.h"

namespace nz {

hipError_t launch_clear(const NzSample *desc, const int32_t *list, int32_t nsamp, uint8_t *ws, NzState *state,
                        hipStream_t st)
{
    if (nsamp <= 0) return hipSuccess;
    hipLaunchKernelGGL(nz_clear_kernel, dim3(nsamp), dim3(256), 0, st, desc, list, nsamp, ws, state);
    return hipGetLastError();
}

hipError_t launch_keys(const NzSample *desc, const int32_t *list, int32_t first, int32_t count, int32_t N, uint8_t *ws,
                       NzState *state, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int32_t bps = (N + KEYS_SITES_PER_BLOCK - 1) / KEYS_SITES_PER_BLOCK;
    const int64_t blocks = static_cast<int64_t>(bps) * count;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(nz_keys_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(KEYS_THREADS), 0, st, desc, list, first,
                       bps, ws, state);
    return hipGetLastError();
}

int32_t keys_sites_per_block() { return KEYS_SITES_PER_BLOCK; }

hipError_t launch_sort(const NzSample *desc, int32_t nsamp, int32_t max_nb, int32_t max_cap, uint8_t *ws,
                       hipStream_t st)
{
    if (nsamp <= 0 || max_nb <= 0) return hipSuccess;
    uint32_t P = 1;
    while (P < static_cast<uint32_t>(max_cap)) P <<= 1;
    const size_t lds = static_cast<size_t>(P) * (sizeof(uint64_t) + sizeof(uint32_t));
    const int64_t items = static_cast<int64_t>(nsamp) * max_nb;
    const uint32_t grid = static_cast<uint32_t>(items < 65536 * 4 ? items : 65536 * 4);
    hipLaunchKernelGGL(nz_sort_kernel, dim3(grid), dim3(SORT_THREADS), lds, st, desc, nsamp, max_nb, ws);
    return hipGetLastError();
}

hipError_t launch_prefill(const NzSample *desc, const int32_t *list, int32_t nlist, int32_t bx_hook, int32_t bx_site,
                          const NzOffset *tabs, uint8_t *ws, NzState *state, hipStream_t st)
{
    if (nlist <= 0) return hipSuccess;
    hipLaunchKernelGGL(nz_hook_kernel, dim3(bx_hook, nlist), dim3(256), 0, st, desc, list, tabs, ws, state);
    hipLaunchKernelGGL(nz_compress_kernel, dim3(bx_site, nlist), dim3(256), 0, st, desc, list, ws, state);
    hipLaunchKernelGGL(nz_accum_kernel, dim3(bx_site, nlist), dim3(256), 0, st, desc, list, ws, state);
    return hipGetLastError();
}

template <int NCH, int RES>
static hipError_t launch_sweep_t(const NzSweepArgs &a, const SweepOut &o, int grid, int wg_waves, size_t lds,
                                 hipStream_t st)
{
    auto k = nz_sweep_kernel<NCH, RES>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * wg_waves), lds, st, a, o);
    return hipGetLastError();
}

template <int RES>
static hipError_t launch_sweep_r(int nch, const NzSweepArgs &a, const SweepOut &o, int grid, int wg_waves, size_t lds,
                                 hipStream_t st)
{
    switch (nch) {
    case 1: return launch_sweep_t<1, RES>(a, o, grid, wg_waves, lds, st);
    case 2: return launch_sweep_t<2, RES>(a, o, grid, wg_waves, lds, st);
    case 4: return launch_sweep_t<4, RES>(a, o, grid, wg_waves, lds, st);
    case 8: return launch_sweep_t<8, RES>(a, o, grid, wg_waves, lds, st);
    case 14: return launch_sweep_t<14, RES>(a, o, grid, wg_waves, lds, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep(int nch, int residency, const NzSweepArgs &a, int32_t *nstar, int32_t *mass,
                        const int32_t *out_index, int grid, int wg_waves, hipStream_t st)
{
    SweepOut o{nstar, mass, out_index};
    const size_t lds = static_cast<size_t>(a.lds_words) * 4u * static_cast<size_t>(wg_waves);
    switch (residency) {
    case RES_HBM: return launch_sweep_r<RES_HBM>(nch, a, o, grid, wg_waves, lds, st);
    case RES_OCC: return launch_sweep_r<RES_OCC>(nch, a, o, grid, wg_waves, lds, st);
    case RES_ALL: return launch_sweep_r<RES_ALL>(nch, a, o, grid, wg_waves, lds, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nz
