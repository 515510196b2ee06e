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
//   nz_hook/label      bulk connected components of the prefilled sites
//   kernels            (hooking with CAS links, then every member points at its
//                      root and adds its size and border flags to the root
//                      word); a state that already spans is flagged for
//                      backoff;
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

// 32x32 -> 64-bit product as one v_mad_u64_u32 (left to itself the compiler
// forms the last round's products with separate v_mul_hi_u32 / v_mul_lo_u32,
// two more quarter-rate instructions per Philox block).
__device__ __forceinline__ uint64_t mul_wide(uint32_t x, uint32_t m)
{
    uint64_t r, carry;
    asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(r), "=&s"(carry) : "v"(x), "s"(m));
    (void)carry;
    return r;
}

// Three-input XOR in one gfx950 instruction (v_bitop3_b32, truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Keys of sites 2j and 2j + 1: both come from the block of counter j (word 3:
// domain tag 0); the even site takes words (1, 0), the odd site words (3, 2).
// Each round's two 32x32 products are formed as full 64-bit products (one
// v_mad_u64_u32 each) and each of its two three-way XORs is one instruction.
__device__ __forceinline__ void site_key_pair(uint32_t seed_lo, uint32_t seed_hi, uint32_t smp_lo, uint32_t smp_hi,
                                              uint32_t j, uint64_t &k_even, uint64_t &k_odd)
{
    uint32_t c0 = j, c1 = smp_lo, c2 = smp_hi, c3 = 0u;
    uint32_t k0 = seed_lo, k1 = seed_hi;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = mul_wide(c0, kPhiloxMulA);
        // round 0's c2 is the sample's high word, the same in every lane
        const uint64_t b = r == 0 ? static_cast<uint64_t>(kPhiloxMulB) * c2 : mul_wide(c2, kPhiloxMulB);
        c0 = xor3(static_cast<uint32_t>(b >> 32), c1, k0);
        c1 = static_cast<uint32_t>(b);
        c2 = xor3(static_cast<uint32_t>(a >> 32), c3, k1);
        c3 = static_cast<uint32_t>(a);
        k0 += kWeylA;
        k1 += kWeylB;
    }
    k_even = (static_cast<uint64_t>(c1) << 32) | c0;
    k_odd = (static_cast<uint64_t>(c3) << 32) | c2;
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

// Periodic boundaries: the index correction of an offset whose steps leave
// the lattice on the axes of `out` (the offset's code bits outside the allowed
// set): +L^(j+1) for a negative step that left through 0, -L^(j+1) for a
// positive one past L-1 (one wrap suffices for L >= 5).
__device__ __forceinline__ int32_t wrap_fix(uint32_t out, int32_t L)
{
    int32_t fix = 0, p = L;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const uint32_t b = (out >> (5 * j)) & 31u;
        fix += (b & 0x03u) ? p : 0;
        fix -= (b & 0x18u) ? p : 0;
        p *= L;
    }
    return fix;
}

// An offset code with bits above 25 marks a padding slot (no offset).
constexpr uint32_t kCodeBits = 0x1FFFFFFu;

// Relaxed wavefront-scope accesses: ordinary cached loads and stores that the
// compiler neither merges nor elides.  They serve state private to one wave and
// the cache-tolerant walks of the bulk connected components; links and counts
// shared by all workgroups use agent-scope atomics.
template <typename T>
__device__ __forceinline__ T ld_w(T *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT); }
template <typename T>
__device__ __forceinline__ void st_w(T *p, T v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT); }

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
    uint32_t *sum = reinterpret_cast<uint32_t *>(ws + d.off_sum);
    for (int w = threadIdx.x; w < d.sum_words; w += blockDim.x) sum[w] = 0u;
    if (threadIdx.x == 0) {
        NzState s;
        s.status = NZ_ST_PENDING;
        s.nstar = 0;
        s.mass = 0;
        s.n0 = 0;
        s.smax = 0;
        state[sid] = s;
    }
}

// ---------------------------------------------------------------------------
// Keys, prefill occupancy and band bucketing.  A block covers
// KEYS_THREADS * 2 * KEYS_ITERS consecutive sites of one sample, wave w the
// KEYS_WAVE_SITES sites from w * KEYS_WAVE_SITES; per iteration a wave takes
// 128 consecutive sites, lane l the pair (2l, 2l + 1) that shares one Philox
// block, so two ballots yield four bitset words.  Lane `it` keeps iteration
// it's ballots; after the loop lane l builds word l & 3 of iteration 16 g +
// l / 4 for every group g of 16 iterations, so the bit interleave runs once for
// all of a wave's words.  A wave's fixed costs (its sample's descriptor, the
// list atomic, the scans) are paid once per KEYS_WAVE_SITES sites: with 1024,
// 2048, 4096 and 8192 sites per wave the kernel alone took 2.99, 1.97, 1.77
// and 1.71 ms for 2000 samples of L = 16, zones 1-7, and 6.72, 4.58, 3.43 and
// 2.88 ms for zone 1.

constexpr int KEYS_THREADS = 256;
#ifndef NZ_KEYS_ITERS
#define NZ_KEYS_ITERS 64
#endif
constexpr int KEYS_ITERS = NZ_KEYS_ITERS;
constexpr int KEYS_WAVE_SITES = 128 * KEYS_ITERS;
constexpr int KEYS_GROUPS = KEYS_ITERS / 16;   // groups of 64 bitset words in a wave's range
constexpr int KEYS_SITES_PER_BLOCK = KEYS_THREADS * 2 * KEYS_ITERS;
static_assert(KEYS_ITERS % 16 == 0 && KEYS_ITERS <= 64, "whole 64-word groups; lane it keeps iteration it");
static_assert(KEYS_SITES_PER_BLOCK == (KEYS_THREADS / 64) * KEYS_WAVE_SITES, "waves tile the block");

// Predicate code of an unsigned less-than for the lane-mask compare builtins.
constexpr int kIcmpUlt = 36;

// The 16 bits of x moved to the even bit positions of a 32-bit word.
__device__ __forceinline__ uint32_t spread_even(uint32_t x)
{
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

struct KeysCtx {
    uint64_t T0;
    int32_t shift;
    uint64_t nb;
    uint32_t cap;
    uint32_t L;
    uint64_t magic;
    int32_t *par;
    uint64_t *keys;
    uint32_t *sites;
    uint32_t *counts;
};

// Band sites of a wave are queued in LDS and bucketed 64 at a time, one per
// lane, so the bucketing work runs on full waves although only a few percent of
// the sites fall into the band.
constexpr uint32_t KEYS_BQ = 192;   // queue entries per wave (< 64 left + 128 new)

__device__ __forceinline__ void keys_bucket(const KeysCtx &c, uint64_t K, uint32_t i)
{
    const uint64_t b = (K - c.T0) >> c.shift;
    const uint32_t slot = atomicAdd(&c.counts[b], 1u);
    if (slot < c.cap) {
        c.keys[b * c.cap + slot] = K;
        c.sites[b * c.cap + slot] = pack_coords(i, c.L, c.magic);
    }
}

// The iterations of one wave over a block: keys, the prefill and band masks,
// the prefill ballots (lane it keeps iteration it's) and the band queue.
// FULL: the block lies wholly inside the lattice (no site needs a range test);
// BALL: the band reaches 2^64 (every key at or above T0 is in it); HI: T0 and
// the band's end are multiples of 2^32, so comparing high words decides.
struct KeysIter {
    const KeysCtx &c;
    uint64_t *qk;
    uint32_t *qs;
    uint32_t N;
    uint32_t wave_base;
    uint32_t lane;
    uint64_t band_end;
    uint32_t seed_lo, seed_hi, smp_lo, smp_hi;
};

template <bool FULL, bool BALL, bool HI>
__device__ __forceinline__ void keys_iters(const KeysIter &k, uint32_t &be_lo, uint32_t &be_hi, uint32_t &bo_lo,
                                           uint32_t &bo_hi, int &its, uint32_t &nq)
{
    const KeysCtx &c = k.c;
    uint64_t *qk = k.qk;
    uint32_t *qs = k.qs;
    const uint32_t lane = k.lane, lane2 = 2u * k.lane;
    for (int it = 0; it < KEYS_ITERS; ++it) {
        const uint32_t wbase = k.wave_base + static_cast<uint32_t>(it) * 128u;   // (scalar)
        if (wbase >= k.N) break;
        its = it + 1;
        uint64_t K0, K1;
        site_key_pair(k.seed_lo, k.seed_hi, k.smp_lo, k.smp_hi, (wbase >> 1) + lane, K0, K1);
        // lane masks of the compares (prefilled: key < T0; band: T0 <= key <
        // band_end), combined on the scalar unit
        const uint64_t vm0 = FULL ? ~0ull : __builtin_amdgcn_uicmp(wbase + lane2, k.N, kIcmpUlt);
        const uint64_t vm1 = FULL ? ~0ull : __builtin_amdgcn_uicmp(wbase + lane2 + 1u, k.N, kIcmpUlt);
        uint64_t be, bo, qe, qo;
        if constexpr (HI) {
            // T0 and band_end are multiples of 2^32: the keys' high words decide
            const uint32_t h0 = static_cast<uint32_t>(K0 >> 32), h1 = static_cast<uint32_t>(K1 >> 32);
            const uint32_t t0 = static_cast<uint32_t>(c.T0 >> 32), te = static_cast<uint32_t>(k.band_end >> 32);
            be = vm0 & __builtin_amdgcn_uicmp(h0, t0, kIcmpUlt);
            bo = vm1 & __builtin_amdgcn_uicmp(h1, t0, kIcmpUlt);
            qe = (vm0 & ~be) & (BALL ? ~0ull : __builtin_amdgcn_uicmp(h0, te, kIcmpUlt));
            qo = (vm1 & ~bo) & (BALL ? ~0ull : __builtin_amdgcn_uicmp(h1, te, kIcmpUlt));
        } else {
            be = vm0 & __builtin_amdgcn_uicmpl(K0, c.T0, kIcmpUlt);
            bo = vm1 & __builtin_amdgcn_uicmpl(K1, c.T0, kIcmpUlt);
            qe = (vm0 & ~be) & (BALL ? ~0ull : __builtin_amdgcn_uicmpl(K0, k.band_end, kIcmpUlt));
            qo = (vm1 & ~bo) & (BALL ? ~0ull : __builtin_amdgcn_uicmpl(K1, k.band_end, kIcmpUlt));
        }
        if (lane == static_cast<uint32_t>(it)) {
            be_lo = static_cast<uint32_t>(be);
            be_hi = static_cast<uint32_t>(be >> 32);
            bo_lo = static_cast<uint32_t>(bo);
            bo_hi = static_cast<uint32_t>(bo >> 32);
        }
        // band: queued, then bucketed in full waves
        const uint32_t nqe = static_cast<uint32_t>(__popcll(qe));
        if (qe) {
            if (__builtin_amdgcn_inverse_ballot_w64(qe)) {
                const uint32_t e = nq + __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(qe >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(qe), 0u));
                qk[e] = K0;
                qs[e] = wbase + lane2;
            }
        }
        if (qo) {
            if (__builtin_amdgcn_inverse_ballot_w64(qo)) {
                const uint32_t e = nq + nqe + __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(qo >> 32),
                                                                        __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(qo), 0u));
                qk[e] = K1;
                qs[e] = wbase + lane2 + 1u;
            }
        }
        nq = __builtin_amdgcn_readfirstlane(nq + nqe + static_cast<uint32_t>(__popcll(qo)));
        __builtin_amdgcn_wave_barrier();
        if (nq >= 64u) {
            uint32_t base = 0;
            for (; base + 64u <= nq; base += 64u) keys_bucket(c, qk[base + lane], qs[base + lane]);
            // move the remainder (< 64 entries) to the front
            const uint32_t rest = nq - base;
            uint64_t rk = 0;
            uint32_t rs = 0;
            if (lane < rest) {
                rk = qk[base + lane];
                rs = qs[base + lane];
            }
            __builtin_amdgcn_wave_barrier();
            if (lane < rest) {
                qk[lane] = rk;
                qs[lane] = rs;
            }
            __builtin_amdgcn_wave_barrier();
            nq = __builtin_amdgcn_readfirstlane(rest);
        }
    }
}

__device__ __forceinline__ void keys_block(const NzSample *__restrict__ desc, const int32_t *__restrict__ list,
                                           int32_t first, int32_t blocks_per_sample, uint8_t *__restrict__ ws,
                                           NzState *__restrict__ state, int32_t vblock)
{
    // Every wave works alone on its own KEYS_WAVE_SITES consecutive sites: no
    // workgroup barrier, so a wave that waits for its list atomic or its
    // sample's descriptor leaves the SIMD to the others.  The wave's prefilled
    // sites are appended to the sample's list in site order with one global
    // atomic, and every bitset word's list position is stored, so that a
    // site's list position is that of its word plus the set bits below it.
    __shared__ uint64_t bq_key[KEYS_THREADS / 64][KEYS_BQ];
    __shared__ uint32_t bq_site[KEYS_THREADS / 64][KEYS_BQ];
    const int which = vblock / blocks_per_sample;
    const int sid = list ? list[first + which] : first + which;
    const int blk = vblock % blocks_per_sample;
    const NzSample &d = desc[sid];
    const uint32_t N = static_cast<uint32_t>(d.N);
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x >> 6;
    // the first site of the wave's range (a multiple of 2048, so its bitset
    // words start on a 64-word boundary)
    const uint32_t wave_base =
        __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(blk) * KEYS_SITES_PER_BLOCK + KEYS_WAVE_SITES * wave);
    if (wave_base >= N) return;   // wave-uniform
    const uint32_t seed_lo = static_cast<uint32_t>(d.seed), seed_hi = static_cast<uint32_t>(d.seed >> 32);
    const uint32_t smp_lo = static_cast<uint32_t>(d.sample), smp_hi = static_cast<uint32_t>(d.sample >> 32);
    const uint32_t occ_words = ((N + 63u) >> 6) << 1;   // padded to whole 64-site words

    KeysCtx c;
    c.T0 = d.T0;
    c.shift = d.shift;
    c.nb = static_cast<uint64_t>(d.nb);
    c.cap = static_cast<uint32_t>(d.cap);
    c.L = static_cast<uint32_t>(d.L);
    c.magic = d.magic;
    c.par = reinterpret_cast<int32_t *>(ws + d.off_par);
    c.keys = reinterpret_cast<uint64_t *>(ws + d.off_keys);
    c.sites = reinterpret_cast<uint32_t *>(ws + d.off_sites);
    c.counts = reinterpret_cast<uint32_t *>(ws + d.off_counts);
    uint32_t *occ = reinterpret_cast<uint32_t *>(ws + d.off_occ);
    uint32_t *prefix = reinterpret_cast<uint32_t *>(ws + d.off_prefix);
    // keys in [T0, band_end) fall into the band (band_end saturates at 2^64)
    const uint64_t span = c.nb << c.shift;
    const bool band_all = c.shift >= 64 || (span >> c.shift) != c.nb || c.T0 + span < c.T0;
    const uint64_t band_end = c.T0 + span;

    uint64_t *qk = bq_key[wave];
    uint32_t *qs = bq_site[wave];
    uint32_t nq = 0;        // wave-uniform
    // wave-uniform choices held in scalar registers: whether the wave's range
    // lies wholly inside the lattice (then no site needs a range test) and
    // whether the band reaches 2^64
    const bool full = __builtin_amdgcn_readfirstlane(wave_base + KEYS_WAVE_SITES <= N ? 1u : 0u) != 0u;
    const bool ball = __builtin_amdgcn_readfirstlane(band_all ? 1u : 0u) != 0u;
    // thresholds on 2^32 boundaries (the planner's choice): 32-bit compares
    const bool hi = __builtin_amdgcn_readfirstlane(
                        ((c.T0 | (band_all ? 0ull : band_end)) & 0xFFFFFFFFull) == 0ull ? 1u : 0u) != 0u;
    // even / odd prefill ballots of iteration it, held by lane it
    uint32_t be_lo = 0, be_hi = 0, bo_lo = 0, bo_hi = 0;
    int its = 0;            // iterations this wave ran (wave-uniform)
    // the loop is compiled for each combination of the two wave-uniform
    // choices, so that no iteration tests them
    KeysIter ki{c, qk, qs, N, wave_base, lane, band_end, seed_lo, seed_hi, smp_lo, smp_hi};
    if (hi) {
        if (full) {
            if (ball) keys_iters<true, true, true>(ki, be_lo, be_hi, bo_lo, bo_hi, its, nq);
            else keys_iters<true, false, true>(ki, be_lo, be_hi, bo_lo, bo_hi, its, nq);
        } else {
            if (ball) keys_iters<false, true, true>(ki, be_lo, be_hi, bo_lo, bo_hi, its, nq);
            else keys_iters<false, false, true>(ki, be_lo, be_hi, bo_lo, bo_hi, its, nq);
        }
    } else if (full) {
        if (ball) keys_iters<true, true, false>(ki, be_lo, be_hi, bo_lo, bo_hi, its, nq);
        else keys_iters<true, false, false>(ki, be_lo, be_hi, bo_lo, bo_hi, its, nq);
    } else {
        if (ball) keys_iters<false, true, false>(ki, be_lo, be_hi, bo_lo, bo_hi, its, nq);
        else keys_iters<false, false, false>(ki, be_lo, be_hi, bo_lo, bo_hi, its, nq);
    }
    if (lane < nq) keys_bucket(c, qk[lane], qs[lane]);

    // Word q of iteration it (sites wave_base + 128 it .. + 127) interleaves
    // bits 16q .. 16q + 15 of the even and odd ballots.  The range's words come
    // in groups of 64, one word per lane: lane l of group g builds word 64 g + l,
    // that of iteration 16 g + l / 4.  Words of iterations that did not run are
    // zero; words past the padded bitset are not stored.
    const uint32_t q = lane & 3u;
    const uint32_t w0 = wave_base >> 5;
    uint32_t word[KEYS_GROUPS];
    bool mine[KEYS_GROUPS];
#pragma unroll
    for (int g = 0; g < KEYS_GROUPS; ++g) {
        const int src = 16 * g + static_cast<int>(lane >> 2);
        const uint32_t elo = static_cast<uint32_t>(__shfl(static_cast<int>(be_lo), src));
        const uint32_t ehi = static_cast<uint32_t>(__shfl(static_cast<int>(be_hi), src));
        const uint32_t olo = static_cast<uint32_t>(__shfl(static_cast<int>(bo_lo), src));
        const uint32_t ohi = static_cast<uint32_t>(__shfl(static_cast<int>(bo_hi), src));
        const uint32_t sh = 16u * (q & 1u);
        const uint32_t e16 = ((q < 2u ? elo : ehi) >> sh) & 0xFFFFu;
        const uint32_t o16 = ((q < 2u ? olo : ohi) >> sh) & 0xFFFFu;
        mine[g] = src < its;
        word[g] = mine[g] ? (spread_even(e16) | (spread_even(o16) << 1)) : 0u;
        const uint32_t w = w0 + 64u * static_cast<uint32_t>(g) + lane;
        if (mine[g] && w < occ_words) occ[w] = word[g];
    }
    if (d.T0 == 0) return;   // plain sample: nothing prefilled (uniform over the grid)

    // summary bits of the range's non-empty words, and the exclusive scan of
    // the word counts of every group
    uint32_t *sum = reinterpret_cast<uint32_t *>(ws + d.off_sum);
    const uint32_t gs = static_cast<uint32_t>(d.sum_shift);
    uint32_t wc[KEYS_GROUPS], excl[KEYS_GROUPS], cnt[KEYS_GROUPS];
    uint32_t total = 0;
#pragma unroll
    for (int g = 0; g < KEYS_GROUPS; ++g) {
        wc[g] = static_cast<uint32_t>(__popc(word[g]));
        const uint32_t wg0 = w0 + 64u * static_cast<uint32_t>(g);   // a multiple of 64
        if (d.sum_words > 0) {
            const uint64_t nzw = __ballot(wc[g] != 0u);
            if (gs == 0u) {
                // one bit per word: the group's bits fill two whole words
                const uint32_t half = lane < 2u ? static_cast<uint32_t>(nzw >> (32u * lane)) : 0u;
                if (half) atomicOr(&sum[(wg0 >> 5) + lane], half);
            } else if (lane == 0u && nzw) {
                // bit j of v: any of the 2^gs words j << gs .. of the group (1 <=
                // gs <= 4); k is a multiple of 64 >> gs, so v fits in one word
                const uint32_t span_bits = 64u >> gs;
                const uint64_t grp = (1ull << (1u << gs)) - 1ull;
                uint32_t v = 0u;
                for (uint32_t j = 0; j < span_bits; ++j)
                    if ((nzw >> (j << gs)) & grp) v |= 1u << j;
                const uint32_t k = wg0 >> gs;
                atomicOr(&sum[k >> 5], v << (k & 31u));
            }
        }
        uint32_t incl = wc[g];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = static_cast<uint32_t>(__shfl_up(static_cast<int>(incl), o));
            if (lane >= static_cast<uint32_t>(o)) incl += v;
        }
        excl[g] = incl - wc[g];
        cnt[g] = __builtin_amdgcn_readlane(incl, 63);
        total += cnt[g];
    }
    if (total == 0u) return;   // wave-uniform
    uint32_t got = 0u;
    if (lane == 0u) got = atomicAdd(reinterpret_cast<uint32_t *>(&state[sid].n0), total);
    uint32_t base = __builtin_amdgcn_readlane(got, 0);
    uint32_t *wpos = reinterpret_cast<uint32_t *>(ws + d.off_wpos);
    const uint32_t cap = static_cast<uint32_t>(d.prefix_cap);
    int32_t *parc = reinterpret_cast<int32_t *>(ws + d.off_parc);
#pragma unroll
    for (int g = 0; g < KEYS_GROUPS; ++g) {
        const uint32_t w = w0 + 64u * static_cast<uint32_t>(g) + lane;
        uint32_t pos = base + excl[g];
        if (!d.wrap && mine[g] && w < occ_words) wpos[w] = pos;
        // the word's sites in bit order, one lane per word
        uint32_t bits = word[g];
        const uint32_t site0 = w << 5;
        while (bits) {
            const uint32_t sidx = site0 + static_cast<uint32_t>(__builtin_ctz(bits));
            bits &= bits - 1u;
            if (pos < cap) {
                prefix[pos] = sidx;
                // parent = itself (periodic first-wrap: lattice entry, displacement 0)
                if (d.wrap) reinterpret_cast<uint64_t *>(c.par)[sidx] = sidx;
                else parc[pos] = static_cast<int32_t>(pos);
            }
            ++pos;
        }
        base += cnt[g];
    }
}

// Workgroup g takes the blocks g, g + gridDim.x, ... of the launch (one pass
// when the grid has a workgroup per block).
__global__ __launch_bounds__(KEYS_THREADS) void nz_keys_kernel(const NzSample *__restrict__ desc,
                                                               const int32_t *__restrict__ list, int32_t first,
                                                               int32_t blocks_per_sample, int32_t nblocks,
                                                               uint8_t *__restrict__ ws, NzState *__restrict__ state)
{
    for (int32_t vb = static_cast<int32_t>(blockIdx.x); vb < nblocks; vb += static_cast<int32_t>(gridDim.x)) {
        keys_block(desc, list, first, blocks_per_sample, ws, state, vb);
    }
}

// ---------------------------------------------------------------------------
// Bucket sort: one wave per (sample, bucket); bitonic network in the wave's
// LDS slice over (key, packed site) pairs padded to a power of two, each lane
// taking whole compare-exchange pairs, stages ordered by the wave's own LDS
// ordering (no workgroup barrier); sorted packed sites are written back in
// place.  Over-full buckets are left alone (the sweep reports them if it
// reaches one).

constexpr int SORT_THREADS = 256;

__device__ __forceinline__ bool pair_greater(uint64_t ka, uint32_t pa, uint64_t kb, uint32_t pb)
{
    return ka > kb || (ka == kb && pa > pb);
}

// slice: LDS entries per wave (a power of two >= every bucket's capacity)
__global__ __launch_bounds__(SORT_THREADS) void nz_sort_kernel(const NzSample *__restrict__ desc, int32_t nsamp,
                                                               int32_t max_nb, uint32_t slice, uint8_t *__restrict__ ws)
{
    extern __shared__ uint64_t sort_lds[];
    const uint32_t lane = lane_id();
    const uint32_t waves = blockDim.x >> 6;
    const uint32_t wave = threadIdx.x >> 6;
    uint64_t *k = sort_lds + static_cast<size_t>(wave) * slice;
    uint32_t *p = reinterpret_cast<uint32_t *>(sort_lds + static_cast<size_t>(waves) * slice) + static_cast<size_t>(wave) * slice;
    const uint32_t items = static_cast<uint32_t>(nsamp) * static_cast<uint32_t>(max_nb);
    for (uint32_t item = blockIdx.x * waves + wave; item < items; item += gridDim.x * waves) {
        const int sid = static_cast<int>(item / static_cast<uint32_t>(max_nb));
        const int b = static_cast<int>(item - static_cast<uint32_t>(sid) * static_cast<uint32_t>(max_nb));
        const NzSample &d = desc[sid];
        if (b >= d.nb) continue;
        const uint32_t *counts = reinterpret_cast<const uint32_t *>(ws + d.off_counts);
        const uint32_t cnt = counts[b];
        const uint32_t cap = static_cast<uint32_t>(d.cap);
        if (cnt <= 1u || cnt > cap) continue;
        uint32_t P = 2;
        while (P < cnt) P <<= 1;
        const uint64_t *gk = reinterpret_cast<const uint64_t *>(ws + d.off_keys) + static_cast<uint64_t>(b) * cap;
        uint32_t *gp = reinterpret_cast<uint32_t *>(ws + d.off_sites) + static_cast<uint64_t>(b) * cap;
        for (uint32_t i = lane; i < P; i += 64u) {
            if (i < cnt) {
                k[i] = gk[i];
                p[i] = gp[i];
            } else {
                k[i] = ~0ull;
                p[i] = ~0u;
            }
        }
        __builtin_amdgcn_wave_barrier();
        const uint32_t half = P >> 1;
        for (uint32_t size = 2; size <= P; size <<= 1) {
            for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                // pair q: i has bit `stride` clear, j = i + stride
                for (uint32_t q = lane; q < half; q += 64u) {
                    const uint32_t i = ((q & ~(stride - 1u)) << 1) | (q & (stride - 1u));
                    const uint32_t j = i | stride;
                    const bool up = (i & size) == 0u;
                    const uint64_t ki = k[i], kj = k[j];
                    const uint32_t pi = p[i], pj = p[j];
                    if (pair_greater(ki, pi, kj, pj) == up) {
                        k[i] = kj; k[j] = ki;
                        p[i] = pj; p[j] = pi;
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        for (uint32_t i = lane; i < cnt; i += 64u) gp[i] = p[i];
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------------------
// Bulk connected components of the prefilled sites (hook, then label).
// During this phase par[i] is a plain parent index and a root points to
// itself.  Every link goes from a larger index to a smaller one, and only an
// agent-scope CAS that finds par[u] == u links u, so along every path indices
// decrease and no cycle can form.  The walks therefore read through the caches
// (wavefront-scope accesses): a stale entry is still an ancestor (or a former
// root), which can only make a CAS fail and retry from the value it returns,
// one true step further up; path-halving writes store an ancestor.

__device__ __forceinline__ int32_t cc_find(int32_t *par, int32_t x)
{
    int32_t p = ld_w(&par[x]);
    while (p != x) {
        const int32_t g = ld_w(&par[p]);
        if (g != p) st_w(&par[x], g);   // halving: x skips to its grandparent
        x = p;
        p = g;
    }
    return x;
}

// Workgroup l of a prefill launch covers block x of sample slot y.  The
// workgroups of one sample share l mod 8, so they are dispatched to the same
// XCD and the sample's bitset and parents stay in that XCD's L2.
__device__ __forceinline__ bool xcd_slot(int32_t nlist, int32_t bx, int32_t &y, int32_t &x)
{
    const uint32_t l = blockIdx.x;
    const uint32_t k = l >> 3;
    y = static_cast<int32_t>((k / static_cast<uint32_t>(bx)) * 8u + (l & 7u));
    x = static_cast<int32_t>(k % static_cast<uint32_t>(bx));
    return y < nlist;
}

// The bulk labelling runs on the prefilled sites' list positions, not on
// lattice indices: parc[i] is the parent of list entry i, so the whole forest
// of a sample is 4 bytes per prefilled site and stays in the L2 of the XCD that
// holds the sample.  The list position of an occupied neighbour t is the
// position of its bitset word (wpos) plus the set bits below t in that word.
// The size pass points the lattice entry of every prefilled site at the list
// node of its cluster's root; the prefilled roots keep their root words in the
// list forest, where the sweep reads and updates them.

// A union-find node id: a lattice site s (< 2^29) or LIST_NODE | i, list entry
// i of the sample's prefilled sites.  Parent entries hold node ids or root
// words (bit 31 set).
constexpr int32_t LIST_NODE = 0x20000000;

// Hook: one lane per prefilled site and its forward half of the offset table
// (one of each +-d pair), eight neighbour words loaded at a time.  The edges a
// wave finds (site, occupied neighbour) are not linked where they are found:
// each offset slot has only a few lanes with an occupied neighbour, so linking
// slot by slot would run one round of dependent finds per slot with most lanes
// idle.  They are appended to a per-wave edge buffer in LDS instead, and the
// buffer is linked 64 edges at a time, every lane with an edge of its own.
constexpr int HOOK_UNROLL = 8;
// edges buffered per wave: one offset slot adds at most 64, and the buffer is
// emptied whenever it holds 64 or more (a small buffer leaves LDS for more
// resident workgroups: this kernel is bound by the latency of its dependent
// loads and atomics)
constexpr int HOOK_EBUF = 128;

// Summary words a hook workgroup stages in LDS (the host sizes summaries to at
// most 1025 words).
constexpr int32_t HOOK_SUM_MAX = 1025;

// Links list positions a and b: CAS links go from the larger root to the
// smaller, only onto an entry that is still a root, retried from the parent the
// CAS returns.
__device__ __forceinline__ void cc_link(int32_t *par, int32_t a, int32_t b)
{
    int32_t u = cc_find(par, a);
    int32_t v = cc_find(par, b);
    while (u != v) {
        const int32_t hi = max(u, v), lo = min(u, v);
        int32_t expected = hi;
        if (__hip_atomic_compare_exchange_strong(&par[hi], &expected, lo, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            break;
        // hi is no longer a root: go on from the parent the CAS returned
        u = cc_find(par, u == hi ? expected : u);
        v = cc_find(par, v == hi ? expected : v);
    }
}

// The buffered edges 0 .. ne-1 of one wave, 64 at a time.
__device__ __forceinline__ void hook_flush(int32_t *par, const int32_t *ei, const int32_t *ej, int32_t ne, uint32_t lane)
{
    for (int32_t e0 = 0; e0 < ne; e0 += 64) {
        const int32_t e = e0 + static_cast<int32_t>(lane);
        if (e < ne) cc_link(par, ld_w(&ei[e]), ld_w(&ej[e]));
    }
}

// PER: periodic coordinates (compiled apart, so that the free-boundary hook
// carries no wrap correction).
template <bool PER>
__global__ __launch_bounds__(256) void nz_hook_kernel(const NzSample *__restrict__ desc, const int32_t *__restrict__ list,
                                                      int32_t nlist, int32_t bx, const NzOffset *__restrict__ tabs,
                                                      uint8_t *__restrict__ ws, NzState *__restrict__ state)
{
    __shared__ uint32_t hsum[HOOK_SUM_MAX];
    __shared__ int32_t ebuf_i[4][HOOK_EBUF];
    __shared__ int32_t ebuf_j[4][HOOK_EBUF];
    int32_t y, x;
    if (!xcd_slot(nlist, bx, y, x)) return;
    const int sid = list[y];
    const NzSample &d = desc[sid];
    const int32_t n0 = state[sid].n0;
    if (n0 > d.prefix_cap || d.wrap || x * 256 >= n0) return;   // (uniform over the workgroup)
    // A sparse prefill (under one site in 32) leaves most bitset words empty:
    // the workgroup stages the bitset summary in LDS and skips the loads of
    // empty words.
    const bool use_sum = d.sum_words > 0 && d.sum_words <= HOOK_SUM_MAX && static_cast<int64_t>(n0) * 32 < d.N;
    if (use_sum) {
        const uint32_t *sum_g = reinterpret_cast<const uint32_t *>(ws + d.off_sum);
        for (int32_t w = static_cast<int32_t>(threadIdx.x); w < d.sum_words; w += 256) hsum[w] = sum_g[w];
    }
    __syncthreads();
    const uint32_t gs = static_cast<uint32_t>(d.sum_shift);
    const int32_t L = d.L;
    const int32_t zh = d.z >> 1;
    const uint64_t magic = d.magic;
    int32_t *par = reinterpret_cast<int32_t *>(ws + d.off_parc);
    const uint32_t *occ = reinterpret_cast<const uint32_t *>(ws + d.off_occ);
    const uint32_t *wpos = reinterpret_cast<const uint32_t *>(ws + d.off_wpos);
    const uint32_t *prefix = reinterpret_cast<const uint32_t *>(ws + d.off_prefix);
    const NzOffset *tab = tabs + d.tab;
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x >> 6;
    int32_t *ei = ebuf_i[wave];
    int32_t *ej = ebuf_j[wave];
    // the wave's 64 sites per pass (wave-uniform loop; lanes past n0 idle)
    for (int32_t ib = x * 256 + static_cast<int32_t>(wave) * 64; ib < n0; ib += bx * 256) {
        const int32_t i = ib + static_cast<int32_t>(lane);
        const bool act = i < n0;
        const int32_t s = act ? static_cast<int32_t>(prefix[i]) : 0;
        const uint32_t pc = pack_coords(static_cast<uint32_t>(s), static_cast<uint32_t>(L), magic);
        const uint32_t A = act ? (allowed_axis(pc & 63, L) | (allowed_axis((pc >> 6) & 63, L) << 5) |
                                  (allowed_axis((pc >> 12) & 63, L) << 10) | (allowed_axis((pc >> 18) & 63, L) << 15) |
                                  (allowed_axis(pc >> 24, L) << 20))
                               : 0u;
        int32_t ne = 0;   // edges in the buffer (wave-uniform)
        for (int32_t k0 = 0; k0 < zh; k0 += HOOK_UNROLL) {
            int32_t t[HOOK_UNROLL];
            uint32_t w[HOOK_UNROLL];
#pragma unroll
            for (int q = 0; q < HOOK_UNROLL; ++q) {
                NzOffset o;
                o.stride = 0;
                o.code = 0xFFFFFFFFu;
                if (k0 + q < zh) o = tab[k0 + q];
                const uint32_t out = o.code & ~A;
                bool ok;
                if constexpr (PER) {
                    ok = act && (o.code & ~kCodeBits) == 0u;   // every offset wraps back in, padding aside
                    t[q] = s + o.stride + (out ? wrap_fix(out, L) : 0);
                } else {
                    ok = act && out == 0u;
                    t[q] = s + o.stride;
                }
                const uint32_t wi = static_cast<uint32_t>(t[q]) >> 5;
                const bool maybe = !use_sum || ((hsum[(wi >> gs) >> 5] >> ((wi >> gs) & 31)) & 1u);
                w[q] = ok && maybe ? occ[wi] : 0u;
            }
            // list positions of the occupied neighbours: their words' first
            // positions, loaded together, plus the set bits below them
            uint32_t jw[HOOK_UNROLL];
#pragma unroll
            for (int q = 0; q < HOOK_UNROLL; ++q)
                jw[q] = ((w[q] >> (t[q] & 31)) & 1u) ? wpos[static_cast<uint32_t>(t[q]) >> 5] : 0xFFFFFFFFu;
#pragma unroll
            for (int q = 0; q < HOOK_UNROLL; ++q) {
                const bool edge = jw[q] != 0xFFFFFFFFu;
                const uint64_t mk = __ballot(edge);
                if (edge) {
                    const int32_t e = ne + static_cast<int32_t>(__builtin_amdgcn_mbcnt_hi(
                                               static_cast<uint32_t>(mk >> 32),
                                               __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mk), 0u)));
                    st_w(&ei[e], i);
                    st_w(&ej[e], static_cast<int32_t>(jw[q] + static_cast<uint32_t>(__popc(w[q] & ((1u << (t[q] & 31)) - 1u)))));
                }
                ne += static_cast<int32_t>(__popcll(mk));
                if (ne >= 64) {
                    __builtin_amdgcn_wave_barrier();
                    hook_flush(par, ei, ej, ne, lane);
                    __builtin_amdgcn_wave_barrier();
                    ne = 0;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        hook_flush(par, ei, ej, ne, lane);
        __builtin_amdgcn_wave_barrier();
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
                                                          int32_t nlist, int32_t bx, uint8_t *__restrict__ ws,
                                                          NzState *__restrict__ state)
{
    int32_t y, x;
    if (!xcd_slot(nlist, bx, y, x)) return;
    const int sid = list[y];
    const NzSample &d = desc[sid];
    const int32_t n0 = state[sid].n0;
    if (n0 > d.prefix_cap || d.wrap) return;
    const uint32_t L = static_cast<uint32_t>(d.L);
    int32_t *par = reinterpret_cast<int32_t *>(ws + d.off_parc);
    const uint32_t *prefix = reinterpret_cast<const uint32_t *>(ws + d.off_prefix);
    for (int32_t k = x * 256 + static_cast<int32_t>(threadIdx.x); k < n0; k += bx * 256) {
        int32_t r = k;
        int32_t p = ld_w(&par[r]);
        while (p >= 0 && p != r) {
            r = p;
            p = ld_w(&par[r]);
        }
        if (r == k) {
            const uint32_t fl = d.periodic ? 0u : border_flags(prefix[k], L, d.magic);
            st_w(&par[k], static_cast<int32_t>(NZ_ROOT | fl | 1u));
            if (fl == NZ_FLAGS) state[sid].status = NZ_ST_BACKOFF;   // L = 1: one site spans
        } else {
            st_w(&par[k], r);
        }
    }
}

// Sizes, border flags and lattice entries of the prefilled sites, in one pass
// over the list: a member adds itself to its root's word in the list forest,
// and the lattice entry of every prefilled site points at the list node of its
// cluster's root (its own node for a root), where the sweep reads and updates
// the root word.  The flag OR returns the previous word, so the member that
// completes a root's pair of border flags sees it: the state already spans and
// the sample backs off (not in largest-cluster runs, which stop below the
// window instead).
__global__ __launch_bounds__(256) void nz_accum_kernel(const NzSample *__restrict__ desc, const int32_t *__restrict__ list,
                                                       int32_t nlist, int32_t bx, uint8_t *__restrict__ ws,
                                                       NzState *__restrict__ state)
{
    int32_t y, x;
    if (!xcd_slot(nlist, bx, y, x)) return;
    const int sid = list[y];
    const NzSample &d = desc[sid];
    if (d.wrap) return;
    const int32_t n0 = state[sid].n0;
    if (n0 > d.prefix_cap) {
        if (x == 0 && threadIdx.x == 0) state[sid].status = NZ_ST_PREFIX;
        return;
    }
    const uint32_t L = static_cast<uint32_t>(d.L);
    int32_t *parc = reinterpret_cast<int32_t *>(ws + d.off_parc);
    int32_t *par = reinterpret_cast<int32_t *>(ws + d.off_par);
    const uint32_t *prefix = reinterpret_cast<const uint32_t *>(ws + d.off_prefix);
    bool spans = false;
    for (int32_t k = x * 256 + static_cast<int32_t>(threadIdx.x); k < n0; k += bx * 256) {
        const int32_t r = parc[k];
        const uint32_t site = prefix[k];
        if (r >= 0) {
            uint32_t *root = reinterpret_cast<uint32_t *>(&parc[r]);
            atomicAdd(root, 1u);
            const uint32_t fl = d.periodic ? 0u : border_flags(site, L, d.magic);
            if (fl) {
                const uint32_t old = atomicOr(root, fl);
                spans = spans || ((old | fl) & NZ_FLAGS) == NZ_FLAGS;
            }
        }
        par[site] = LIST_NODE | (r >= 0 ? r : k);
    }
    if (spans && !d.smax_mode) state[sid].status = NZ_ST_BACKOFF;
}

// Largest cluster of the prefilled state (smax mode): every root word offers
// its size.
__global__ __launch_bounds__(256) void nz_rootmax_kernel(const NzSample *__restrict__ desc,
                                                         const int32_t *__restrict__ list, int32_t nlist, int32_t bx,
                                                         uint8_t *__restrict__ ws, NzState *__restrict__ state)
{
    int32_t y, x;
    if (!xcd_slot(nlist, bx, y, x)) return;
    const int sid = list[y];
    const NzSample &d = desc[sid];
    if (!d.smax_mode) return;
    const int32_t n0 = state[sid].n0;
    if (n0 > d.prefix_cap) return;
    const int32_t *par = reinterpret_cast<const int32_t *>(ws + d.off_parc);
    int32_t best = 0;
    for (int32_t k = x * 256 + static_cast<int32_t>(threadIdx.x); k < n0; k += bx * 256) {
        const int32_t v = par[k];
        if (v < 0) best = max(best, static_cast<int32_t>(static_cast<uint32_t>(v) & NZ_SIZE));
    }
    if (best > 0) atomicMax(&state[sid].smax, best);
}

// Sum over the finished samples of a chunk of their S_max(n) windows (all
// samples of an smax-mode batch share one window of w entries).
__global__ __launch_bounds__(256) void nz_winsum_kernel(const NzSample *__restrict__ desc,
                                                        const NzState *__restrict__ state, int32_t nsamp, int32_t w,
                                                        const uint8_t *__restrict__ ws, uint64_t *__restrict__ out)
{
    for (int32_t i = blockIdx.x * 256 + static_cast<int32_t>(threadIdx.x); i < w; i += gridDim.x * 256) {
        uint64_t sum = 0;
        for (int32_t k = 0; k < nsamp; ++k) {
            if (state[k].status != NZ_ST_DONE) continue;
            sum += reinterpret_cast<const uint32_t *>(ws + desc[k].off_win)[i];
        }
        out[i] += sum;
    }
}

// ---------------------------------------------------------------------------
// The sweep.  RES selects where the per-sample state of the running wave lives:
//   RES_HBM  bitset and parents in the workspace (HBM / L2);
//   RES_OCC  bitset in this wave's LDS slice, parents in HBM;
//   RES_ALL  bitset and parents in LDS.
// NCH = number of 64-offset chunks the kernel is compiled for (z <= 64 * NCH).

enum { RES_HBM = 0, RES_OCC = 1, RES_ALL = 2 };

// With the bitset in HBM, the wave's LDS slice starts with a summary of it:
// bit k is clear only if bitset words k << sshift .. ((k + 1) << sshift) - 1
// are all zero.  An occupancy check reads the summary first and fetches the
// word from HBM only when its bit is set; near the threshold most words of a
// wide neighbourhood's lattice are empty.  Bits are set when sites are added
// and never cleared (a stale set bit only costs a load).
template <int RES>
struct SweepMem {
    uint32_t *occ_g;
    int32_t *par_g;
    int32_t *parc_g;    // the list forest of the prefilled sites (node ids LIST_NODE | i)
    uint32_t lbase;     // first LDS word of this wave's slice
    uint32_t occ_words; // bitset words (padded to 64 sites)
    uint32_t sshift;    // summary: log2 of bitset words per bit
    bool sum_on;        // the summary is in use (RES_HBM only)

    __device__ __forceinline__ bool maybe(uint32_t *lds, uint32_t w) const
    {
        if constexpr (RES != RES_HBM) return true;
        if (!sum_on) return true;
        const uint32_t k = w >> sshift;
        return (ld_w(&lds[lbase + (k >> 5)]) >> (k & 31)) & 1u;
    }
    __device__ __forceinline__ void mark(uint32_t *lds, uint32_t w) const
    {
        if constexpr (RES == RES_HBM) {
            if (sum_on) {
                const uint32_t k = w >> sshift;
                __hip_atomic_fetch_or(&lds[lbase + (k >> 5)], 1u << (k & 31), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
        }
    }
    __device__ __forceinline__ uint32_t occ_ld(uint32_t *lds, uint32_t w) const
    {
        if constexpr (RES == RES_HBM) return maybe(lds, w) ? ld_w(&occ_g[w]) : 0u;
        else return ld_w(&lds[lbase + w]);
    }
    // called by every lane with the same word and value
    __device__ __forceinline__ void occ_st(uint32_t *lds, uint32_t w, uint32_t v) const
    {
        if constexpr (RES == RES_HBM) {
            st_w(&occ_g[w], v);
            if (lane_id() == 0) mark(lds, w);
        } else {
            st_w(&lds[lbase + w], v);
        }
    }
    // several lanes may set bits of one word at once
    __device__ __forceinline__ void occ_or(uint32_t *lds, uint32_t w, uint32_t bits) const
    {
        if constexpr (RES == RES_HBM) {
            __hip_atomic_fetch_or(&occ_g[w], bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            mark(lds, w);
        } else {
            __hip_atomic_fetch_or(&lds[lbase + w], bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
    }
    __device__ __forceinline__ void occ_andn(uint32_t *lds, uint32_t w, uint32_t bits) const
    {
        if constexpr (RES == RES_HBM)
            __hip_atomic_fetch_and(&occ_g[w], ~bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        else
            __hip_atomic_fetch_and(&lds[lbase + w], ~bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    // parent entry of node i (a lattice site, or a list node of the prefill)
    __device__ __forceinline__ int32_t par_ld(uint32_t *lds, int32_t i) const
    {
        if (i >= LIST_NODE) return ld_w(&parc_g[i - LIST_NODE]);
        if constexpr (RES == RES_ALL) return static_cast<int32_t>(ld_w(&lds[lbase + occ_words + i]));
        else return ld_w(&par_g[i]);
    }
    __device__ __forceinline__ void par_st(uint32_t *lds, int32_t i, int32_t v) const
    {
        if (i >= LIST_NODE) {
            st_w(&parc_g[i - LIST_NODE], v);
            return;
        }
        if constexpr (RES == RES_ALL) st_w(&lds[lbase + occ_words + i], static_cast<uint32_t>(v));
        else st_w(&par_g[i], v);
    }
};

// Root of x with path halving, given v = the parent word of x; returns the root
// index and its root word.
template <int RES>
__device__ __forceinline__ void sweep_find_from(const SweepMem<RES> &m, uint32_t *lds, int32_t x, int32_t v,
                                                int32_t &root, uint32_t &word)
{
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

template <int RES>
__device__ __forceinline__ void sweep_find(const SweepMem<RES> &m, uint32_t *lds, int32_t x, int32_t &root, uint32_t &word)
{
    sweep_find_from<RES>(m, lds, x, m.par_ld(lds, x), root, word);
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

// The key band of one sample in (key, site) order: buckets in key order, each
// already sorted; 64 entries are fetched at a time into one register per lane.
struct BandCursor {
    const uint32_t *counts;
    const uint32_t *sites;
    uint32_t cap;
    int32_t nb;
    int32_t b;        // current bucket
    uint32_t cnt;     // entries in it
    uint32_t j;       // next entry
    uint32_t base;    // entry held by lane 0
    uint32_t mine;    // entry base + lane

    __device__ __forceinline__ void init(const uint32_t *c, const uint32_t *s, uint32_t cp, int32_t n)
    {
        counts = c;
        sites = s;
        cap = cp;
        nb = n;
        b = -1;
        cnt = 0;
        j = 0;
        base = 0;
        mine = 0;
    }

    // 1: pc holds the next site; 0: the band is exhausted; -1: the next
    // non-empty bucket overflowed its capacity.
    __device__ __forceinline__ int next(uint32_t &pc, uint32_t lane)
    {
        while (j >= cnt) {
            ++b;
            if (b >= nb) return 0;
            cnt = counts[b];
            if (cnt > cap) return -1;
            j = 0;
            base = 0;
            mine = lane < cnt ? sites[static_cast<uint64_t>(b) * cap + lane] : 0u;
        }
        if (j - base >= 64u) {
            base = j;
            mine = base + lane < cnt ? sites[static_cast<uint64_t>(b) * cap + base + lane] : 0u;
        }
        pc = bcast(mine, static_cast<int>(j - base));
        ++j;
        return 1;
    }
};

// One sequential step's site and the occupancy words of its neighbours (lane
// c*64 + lane holds neighbour c of the offset table).  PER: coordinates wrap
// modulo L (periodic boundaries); a compile-time choice, so that the
// free-boundary step carries no wrap arithmetic.
template <int NCH, bool PER = false>
struct SiteStep {
    int32_t s;
    uint32_t fl;
    uint32_t own;
    uint32_t A;          // allowed axes of s
    uint32_t word[NCH];  // 0 for a neighbour outside the lattice

    // Neighbour c of s (recomputed rather than held: one register per chunk
    // less, which keeps wide-neighbourhood kernels at more waves per SIMD).
    __device__ __forceinline__ int32_t nbr(int c, const int32_t (&ostride)[NCH], const uint32_t (&ocode)[NCH],
                                           int32_t L) const
    {
        if constexpr (PER) {
            const uint32_t out = ocode[c] & ~A;
            return s + ostride[c] + (out ? wrap_fix(out, L) : 0);
        } else {
            return s + ostride[c];
        }
    }
    // neighbour c lies inside the lattice (under periodic boundaries every
    // offset does, padding slots aside)
    __device__ __forceinline__ bool inside(int c, const uint32_t (&ocode)[NCH]) const
    {
        if constexpr (PER) return (ocode[c] & ~kCodeBits) == 0u;
        else return (ocode[c] & ~A) == 0u;
    }

    template <int RES>
    __device__ __forceinline__ void prepare(const SweepMem<RES> &m, uint32_t *lds, uint32_t pc, int32_t L,
                                            const int32_t (&ostride)[NCH], const uint32_t (&ocode)[NCH])
    {
        const int32_t x0 = pc & 63, x1 = (pc >> 6) & 63, x2 = (pc >> 12) & 63, x3 = (pc >> 18) & 63, x4 = pc >> 24;
        s = x0 + L * (x1 + L * (x2 + L * (x3 + L * x4)));
        A = allowed_axis(x0, L) | (allowed_axis(x1, L) << 5) | (allowed_axis(x2, L) << 10) |
            (allowed_axis(x3, L) << 15) | (allowed_axis(x4, L) << 20);
        fl = PER ? 0u : ((x0 == 0 ? NZ_FLO : 0u) | (x0 == L - 1 ? NZ_FHI : 0u));
        own = m.occ_ld(lds, static_cast<uint32_t>(s) >> 5);
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            word[c] = inside(c, ocode) ? m.occ_ld(lds, static_cast<uint32_t>(nbr(c, ostride, ocode, L)) >> 5) : 0u;
    }

    // Account for site p, occupied after these words were loaded.
    __device__ __forceinline__ void patch(int32_t p, const int32_t (&ostride)[NCH], const uint32_t (&ocode)[NCH], int32_t L)
    {
        const uint32_t bit = 1u << (p & 31);
        if ((s >> 5) == (p >> 5)) own |= bit;
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            if (inside(c, ocode) && nbr(c, ostride, ocode, L) == p) word[c] |= bit;
    }
};

// The next site's occupancy is loaded one step ahead only while the doubled
// per-lane arrays stay small (z <= 128); wider neighbourhoods have few
// sequential steps and would spill registers.
template <int NCH>
constexpr bool kLookahead = NCH <= 2;

// One sequential addition: store the site's occupancy bit, find the distinct
// roots of its occupied neighbours (lanes 0..D-1 hold them, entry 0 being the
// site itself), and merge them into the largest.  Returns the merged cluster's
// size and border flags.
template <int NCH, int RES, bool PER>
__device__ __forceinline__ void sweep_step(const SweepMem<RES> &m, uint32_t *lds, const SiteStep<NCH, PER> &cur,
                                           const int32_t (&ostride)[NCH], const uint32_t (&ocode)[NCH], int32_t L,
                                           int dcap, uint32_t &total, uint32_t &flags)
{
    const uint32_t lane = lane_id();
    const int32_t s = cur.s;
    // all lanes store the same updated word of s (this wave is the only writer
    // of the sample's bitset)
    m.occ_st(lds, static_cast<uint32_t>(s) >> 5, cur.own | (1u << (s & 31)));

    int32_t lroot = s;
    uint32_t lword = NZ_ROOT | cur.fl | 1u;
    int D = 1;
    // Enter the roots found by the lanes of mk (root / rw) into the list.
    auto enter = [&](uint64_t mk, int32_t root, uint32_t rw) {
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
    };
    // Near the threshold a wide neighbourhood has a few occupied neighbours,
    // rarely two on one lane: then every lane holds at most one and all the
    // finds run at once instead of one offset chunk after another.
    int32_t cand = -1;
    bool two = false;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int32_t t = cur.nbr(c, ostride, ocode, L);
        if ((cur.word[c] >> (t & 31)) & 1u) {   // the word is 0 outside the lattice
            two = two || cand >= 0;
            cand = t;
        }
    }
    if (NCH == 1 || !__ballot(two)) {
        const uint64_t mk = __ballot(cand >= 0);
        if (mk) {
            int32_t root = 0;
            uint32_t rw = 0;
            if (cand >= 0) sweep_find<RES>(m, lds, cand, root, rw);
            enter(mk, root, rw);
        }
    } else {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int32_t t = cur.nbr(c, ostride, ocode, L);
            const bool o = (cur.word[c] >> (t & 31)) & 1u;
            const uint64_t mk = __ballot(o);
            if (!mk) continue;
            int32_t root = 0;
            uint32_t rw = 0;
            if (o) sweep_find<RES>(m, lds, t, root, rw);
            enter(mk, root, rw);
        }
    }
    sweep_merge<RES>(m, lds, D, lroot, lword, total, flags);
}

// ---------------------------------------------------------------------------
// Block sweep: the next 64 sites of the order are added by one wave at once,
// one site per lane.  The neighbour checks and root finds of the 64 sites
// overlap in memory instead of following each other; the unions run as a small
// connected-components pass over a graph whose nodes are the block's sites and
// the earlier clusters they touch.  Spanning is monotone in the occupation (a
// cluster only grows and its border flags only accumulate), so if no cluster
// spans after all 64 additions none spanned after any of them and the block is
// committed as a whole.  The single block in which the first spanning cluster
// appears, and blocks that do not fit the tables below, are undone and redone
// one site at a time, which yields the exact n* and mass.
//
// While a block is processed its sites are marked occupied and their parent
// entries hold BLK_MARK | position, a value no node id reaches (sites below
// 2^29, list nodes below 2^30) and no root word has (bit 31 clear).  An occupied neighbour whose parent
// entry carries the mark is a site of the block, earlier or later in the order.
//
// Per-wave LDS slice (32-bit words, at the end of the wave's slice):
//   rkey[256]    open-addressing table of the earlier roots the block touches
//   npar[320]    node parents: node i < 64 is position i, node 64 + h the
//                earlier root in rkey slot h
//   nword[320]   node words in the root-word format (size, flags)

constexpr int BLK_K = 8;               // occupied neighbours recorded per site
constexpr uint32_t BLK_RSLOTS = 256;
constexpr uint32_t BLK_NODES = 64 + BLK_RSLOTS;
constexpr uint32_t BLK_EMPTY = 0xFFFFFFFFu;
constexpr uint32_t BLK_LDS_WORDS = BLK_RSLOTS + 2 * BLK_NODES;
constexpr int BLK_CHUNK = 16;          // neighbour offsets whose loads are issued together
constexpr int32_t BLK_MARK = 0x40000000;

__device__ __forceinline__ uint32_t blk_hash(uint32_t t) { return (t * 0x9E3779B1u) >> 24; }

// Root of node n in the LDS forest, with path halving.  Only non-roots are
// rewritten (to an ancestor), and hooks only change roots, so concurrent finds
// and hooks of the lanes of one wave keep the forest acyclic.
__device__ __forceinline__ uint32_t blk_find(uint32_t *npar, uint32_t x)
{
    for (;;) {
        const uint32_t p = ld_w(&npar[x]);
        if (p == x) return x;
        const uint32_t g = ld_w(&npar[p]);
        if (g == p) return p;
        st_w(&npar[x], g);
        x = g;
    }
}

// Occupied neighbours among BLK_CHUNK offsets (their loads issued together),
// appended to nl[0 .. cntn) by site.
template <int RES>
__device__ __forceinline__ void blk_scan(const SweepMem<RES> &m, uint32_t *lds, const NzOffset (&oq)[BLK_CHUNK],
                                         bool act, int32_t s, uint32_t A, int32_t (&nl)[BLK_K], int &cntn)
{
    int32_t tq[BLK_CHUNK];
    uint32_t wq[BLK_CHUNK];
#pragma unroll
    for (int q = 0; q < BLK_CHUNK; ++q) {
        const bool ok = act && (oq[q].code & ~A) == 0u;
        tq[q] = s + oq[q].stride;
        wq[q] = ok ? m.occ_ld(lds, static_cast<uint32_t>(tq[q]) >> 5) : 0u;
    }
#pragma unroll
    for (int q = 0; q < BLK_CHUNK; ++q) {
        const bool rec = (wq[q] >> (tq[q] & 31)) & 1u;
#pragma unroll
        for (int k = 0; k < BLK_K; ++k) nl[k] = (rec && cntn == k) ? tq[q] : nl[k];
        cntn += rec ? 1 : 0;
    }
}

enum { BLK_COMMITTED = 0, BLK_FALLBACK = 1 };

// Adds the nbk (1..64) sites whose packed coordinates lane i holds in pc (lane
// i = position i of the order); off0 holds the first BLK_CHUNK offsets of the
// table.  BLK_COMMITTED: the block is merged into the union-find and no cluster
// spans.  BLK_FALLBACK: the occupancy bits of the block are cleared again and
// the parents of earlier sites are as before (up to path halving); the caller
// adds the sites one at a time.
template <int RES>
__device__ __forceinline__ int block_step(const SweepMem<RES> &m, uint32_t *lds, uint32_t hbase, int nbk, uint32_t pc,
                                          int32_t L, const NzOffset *tab, const NzOffset (&off0)[BLK_CHUNK], int32_t z,
                                          int max_old)
{
    const uint32_t lane = lane_id();
    const bool act = static_cast<int>(lane) < nbk;
    const int32_t x0 = pc & 63, x1 = (pc >> 6) & 63, x2 = (pc >> 12) & 63, x3 = (pc >> 18) & 63, x4 = pc >> 24;
    const int32_t s = x0 + L * (x1 + L * (x2 + L * (x3 + L * x4)));
    const uint32_t A = allowed_axis(x0, L) | (allowed_axis(x1, L) << 5) | (allowed_axis(x2, L) << 10) |
                       (allowed_axis(x3, L) << 15) | (allowed_axis(x4, L) << 20);
    const uint32_t fl = (x0 == 0 ? NZ_FLO : 0u) | (x0 == L - 1 ? NZ_FHI : 0u);
    uint32_t *rkey = lds + hbase;
    uint32_t *npar = rkey + BLK_RSLOTS;
    uint32_t *nword = npar + BLK_NODES;

    // 1. mark the block's sites (occupied, parent = mark | position); clear
    //    the tables
    if (act) {
        m.par_st(lds, s, BLK_MARK | static_cast<int32_t>(lane));
        m.occ_or(lds, static_cast<uint32_t>(s) >> 5, 1u << (s & 31));
    }
#pragma unroll
    for (uint32_t w = 0; w < BLK_RSLOTS; w += 64) st_w(&rkey[w + lane], BLK_EMPTY);
    for (uint32_t n = lane; n < BLK_NODES; n += 64) st_w(&npar[n], n);
    st_w(&nword[lane], act ? (NZ_ROOT | fl | 1u) : 0u);

    // 2. occupied neighbours (sites of earlier blocks and of this block)
    int32_t nl[BLK_K];
#pragma unroll
    for (int k = 0; k < BLK_K; ++k) nl[k] = 0;
    int cntn = 0;
    blk_scan<RES>(m, lds, off0, act, s, A, nl, cntn);
    for (int c0 = BLK_CHUNK; c0 < z; c0 += BLK_CHUNK) {
        NzOffset oq[BLK_CHUNK];
#pragma unroll
        for (int q = 0; q < BLK_CHUNK; ++q) {
            oq[q].stride = 0;
            oq[q].code = 0xFFFFFFFFu;
            if (c0 + q < z) oq[q] = tab[c0 + q];
        }
        blk_scan<RES>(m, lds, oq, act, s, A, nl, cntn);
    }
    bool bad = cntn > BLK_K;
    __builtin_amdgcn_wave_barrier();

    // 3. parent words of the recorded neighbours (loads issued together).  A
    //    mark names a position of this block: an earlier one becomes an edge to
    //    that node, a later one is dropped.  Otherwise the neighbour's root is
    //    found and entered once into the root table; nl[k] becomes the node
    //    (-1: no edge).
    int32_t pv[BLK_K];
#pragma unroll
    for (int k = 0; k < BLK_K; ++k) pv[k] = (!bad && k < cntn) ? m.par_ld(lds, nl[k]) : -1;
    // the first hop of every find, issued together (a prefilled site points
    // straight at its root, so this usually reaches it)
    int32_t gv[BLK_K];
#pragma unroll
    for (int k = 0; k < BLK_K; ++k) gv[k] = (!bad && k < cntn && pv[k] >= 0 && pv[k] < BLK_MARK) ? m.par_ld(lds, pv[k]) : -1;
    int nnew = 0;
#pragma unroll
    for (int k = 0; k < BLK_K; ++k) {
        if (!bad && k < cntn) {
            if (pv[k] >= BLK_MARK) {
                const int j = pv[k] & 63;
                nl[k] = j < static_cast<int>(lane) ? j : -1;
            } else {
                int32_t root;
                uint32_t word;
                if (pv[k] < 0) {
                    root = nl[k];
                    word = static_cast<uint32_t>(pv[k]);
                } else if (gv[k] < 0) {
                    root = pv[k];
                    word = static_cast<uint32_t>(gv[k]);
                } else {
                    m.par_st(lds, nl[k], gv[k]);   // halving: the neighbour skips to its grandparent
                    sweep_find<RES>(m, lds, gv[k], root, word);
                }
                uint32_t h = blk_hash(static_cast<uint32_t>(root));
                int slot = -1;
                for (uint32_t t = 0; t < BLK_RSLOTS; ++t) {
                    uint32_t expected = BLK_EMPTY;
                    if (__hip_atomic_compare_exchange_strong(&rkey[h], &expected, static_cast<uint32_t>(root),
                                                             __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_WAVEFRONT)) {
                        st_w(&nword[64 + h], word);
                        slot = static_cast<int>(h);
                        ++nnew;
                        break;
                    }
                    if (expected == static_cast<uint32_t>(root)) {
                        slot = static_cast<int>(h);
                        break;
                    }
                    h = (h + 1) & (BLK_RSLOTS - 1);
                }
                bad = bad || slot < 0;
                nl[k] = 64 + slot;
            }
        }
    }
    // the roots entered by all lanes, against the cap on distinct roots
    int nold = nnew;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) nold += __shfl_xor(nold, d);
    if (__ballot(bad) || nold > max_old) {
        if (act) m.occ_andn(lds, static_cast<uint32_t>(s) >> 5, 1u << (s & 31));
        return BLK_FALLBACK;
    }
    __builtin_amdgcn_wave_barrier();

    // 4. connected components: hook the worse root under the better one (larger
    //    size, then larger node), until no edge joins two trees
    for (;;) {
        bool hooked = false;
#pragma unroll
        for (int k = 0; k < BLK_K; ++k) {
            if (k < cntn && nl[k] >= 0) {
                const uint32_t a = blk_find(npar, lane);
                const uint32_t b = blk_find(npar, static_cast<uint32_t>(nl[k]));
                if (a != b) {
                    const uint32_t sa = ld_w(&nword[a]) & NZ_SIZE, sb = ld_w(&nword[b]) & NZ_SIZE;
                    const bool a_up = sa > sb || (sa == sb && a > b);
                    uint32_t expected = a_up ? b : a;
                    __hip_atomic_compare_exchange_strong(&npar[expected], &expected, a_up ? a : b, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                    hooked = true;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (!__ballot(hooked)) break;
    }

    // 5. sizes and flags into the roots; live nodes are the block's positions
    //    and the occupied root-table slots
    uint32_t nroot[BLK_NODES / 64];
    bool nlive[BLK_NODES / 64];
#pragma unroll
    for (uint32_t q = 0; q < BLK_NODES / 64; ++q) {
        const uint32_t n = lane + 64 * q;
        nlive[q] = q == 0 ? act : ld_w(&rkey[n - 64]) != BLK_EMPTY;
        nroot[q] = nlive[q] ? blk_find(npar, n) : n;
        if (nlive[q] && nroot[q] != n) {
            const uint32_t w = ld_w(&nword[n]);
            __hip_atomic_fetch_add(&nword[nroot[q]], w & NZ_SIZE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            __hip_atomic_fetch_or(&nword[nroot[q]], w & NZ_FLAGS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
    }
    __builtin_amdgcn_wave_barrier();
    bool spans = false;
#pragma unroll
    for (uint32_t q = 0; q < BLK_NODES / 64; ++q) {
        const uint32_t n = lane + 64 * q;
        spans = spans || (nlive[q] && nroot[q] == n && (ld_w(&nword[n]) & NZ_FLAGS) == NZ_FLAGS);
    }
    if (__ballot(spans)) {
        if (act) m.occ_andn(lds, static_cast<uint32_t>(s) >> 5, 1u << (s & 31));
        return BLK_FALLBACK;
    }

    // 6. write back: roots get their root word, other nodes link to their root
#pragma unroll
    for (uint32_t q = 0; q < BLK_NODES / 64; ++q) {
        const uint32_t n = lane + 64 * q;
        const uint32_t r = nroot[q];
        const int32_t rsite_pos = __shfl(s, static_cast<int>(r & 63));   // all lanes take part
        if (nlive[q]) {
            const int32_t site = q == 0 ? s : static_cast<int32_t>(ld_w(&rkey[n - 64]));
            int32_t v;
            if (r == n) v = static_cast<int32_t>(ld_w(&nword[n]));
            else v = r < 64 ? rsite_pos : static_cast<int32_t>(ld_w(&rkey[r - 64]));
            m.par_st(lds, site, v);
        }
    }
    return BLK_COMMITTED;
}

struct SweepOut {
    int32_t *nstar;
    int32_t *mass;
    const int32_t *out_index; // per sample: position in the caller's output arrays
};

// NCH: offset chunks of one-site steps; FB: offset chunks of the block
// sweep's one-site fallback (z <= 64 * FB for every block sample), kept
// separate so that a launch whose wide neighbourhoods go one site at a time
// does not carry their registers through the block path.
template <int NCH, int RES, bool BLOCK, int FB, bool PER>
__global__ __launch_bounds__(256) void nz_sweep_kernel(NzSweepArgs a, SweepOut out)
{
    static_assert(!(BLOCK && PER), "periodic samples go one site per step");
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
        m.parc_g = reinterpret_cast<int32_t *>(a.ws + d.off_parc);
        m.lbase = wave * a.lds_words;
        m.occ_words = static_cast<uint32_t>(((N + 63) >> 6) << 1);
        m.sshift = static_cast<uint32_t>(d.sum_shift);
        m.sum_on = false;
        if constexpr (RES == RES_HBM) {
            m.sum_on = a.use_sum != 0 && d.sum_words > 0;
            if (m.sum_on) {
                const uint32_t *sum_g = reinterpret_cast<const uint32_t *>(a.ws + d.off_sum);
                for (int32_t w = lane; w < d.sum_words; w += 64) lds[m.lbase + w] = sum_g[w];
                __builtin_amdgcn_wave_barrier();
            }
        }
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
        // offset c * 64 + lane of the table per lane, for one-site-at-a-time steps
        int32_t ostride[NCH];
        uint32_t ocode[NCH];
        // (relaxed atomic loads: kept where they are rather than hoisted out of
        // the block loop, where the arrays would hold registers for every block)
        auto load_offsets = [&]() {
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int32_t j = c * 64 + static_cast<int32_t>(lane);
                if (j < z) {
                    ostride[c] = ld_w(&tab[j].stride);
                    ocode[c] = ld_w(&tab[j].code);
                } else {
                    ostride[c] = 0;
                    ocode[c] = 0xFFFFFFFFu;   // never inside: bits above 25 are never allowed
                }
            }
        };

        int32_t r = a.state[sid].n0;   // sites already occupied
        int32_t status = NZ_ST_BAND;
        int32_t nstar = 0, mass = 0;
        // smax mode: the sweep runs on past n* and records the largest cluster
        // after every addition with win_lo <= r < win_hi
        const bool smax_mode = d.smax_mode != 0;
        int32_t smax = a.state[sid].smax;
        uint32_t *win = reinterpret_cast<uint32_t *>(a.ws + d.off_win);
        // One addition done (r sites occupied, the new site's cluster has
        // `total` sites and border flags `flags`): true when the sample is over.
        auto finished = [&](uint32_t total, uint32_t flags) -> bool {
            if (flags == NZ_FLAGS && nstar == 0) {
                nstar = r;
                mass = static_cast<int32_t>(total);
                if (!smax_mode) {
                    status = NZ_ST_DONE;
                    return true;
                }
            }
            if (smax_mode) {
                smax = max(smax, static_cast<int32_t>(total));
                if (r >= d.win_lo) win[r - d.win_lo] = static_cast<uint32_t>(smax);   // every lane, same value
                if (r + 1 >= d.win_hi) {
                    status = NZ_ST_DONE;
                    return true;
                }
            }
            return false;
        };

        // 64 sites per step up to the launch's z limit, one site per step above
        // it (and always one at a time in smax mode)
        bool use_block = false;
        if constexpr (BLOCK) use_block = z <= a.blk_zmax && !smax_mode;
        if (smax_mode && r >= d.win_lo) {
            status = NZ_ST_BACKOFF;   // the prefill covers part of the window: start lower
        } else if (use_block) {
            // 64 sites of the band at a time; blocks do not cross buckets
            const uint32_t *counts = reinterpret_cast<const uint32_t *>(a.ws + d.off_counts);
            const uint32_t *sites = reinterpret_cast<const uint32_t *>(a.ws + d.off_sites);
            const uint32_t hbase = m.lbase + a.lds_words - BLK_LDS_WORDS;
            NzOffset off0[BLK_CHUNK];   // the first offsets, kept for the whole sample
#pragma unroll
            for (int q = 0; q < BLK_CHUNK; ++q) {
                off0[q].stride = 0;
                off0[q].code = 0xFFFFFFFFu;
                if (q < z) off0[q] = tab[q];
            }
            SiteStep<FB> cur;
            int32_t fstride[FB];
            uint32_t fcode[FB];
            bool done = false;
            // Block cursor over the band: bucket cb, offset cj of the next site.
            // The concatenated buckets are the order, so a block takes the next
            // 64 sites across bucket boundaries.  Its sites are loaded one block
            // ahead, so that load overlaps the previous block's step.  1: pc
            // holds the block's sites (lanes < n); 0: end of the band; -1: an
            // over-full bucket was reached (the sites before it still form a
            // block first).
            int32_t cb = 0;
            uint32_t cj = 0;
            uint32_t ccnt = nb > 0 ? counts[0] : 0u;
            auto next_block = [&](uint32_t &pc, int &n) -> int {
                n = 0;
                pc = 0u;
                bool over = false;
                while (n < 64) {
                    while (cb < nb && cj >= ccnt) {
                        ++cb;
                        cj = 0;
                        if (cb < nb) ccnt = counts[cb];
                    }
                    if (cb >= nb) break;
                    if (ccnt > cap) {
                        over = true;
                        break;
                    }
                    const uint32_t t = min(static_cast<uint32_t>(64 - n), ccnt - cj);
                    const uint32_t rel = lane - static_cast<uint32_t>(n);   // this lane's entry, if in range
                    if (lane >= static_cast<uint32_t>(n) && rel < t) pc = sites[static_cast<uint64_t>(cb) * cap + cj + rel];
                    n += static_cast<int>(t);
                    cj += t;
                }
                if (n > 0) return 1;
                return over ? -1 : 0;
            };
            uint32_t pcl = 0;
            int nbk = 0;
            int got = next_block(pcl, nbk);
            while (got == 1) {
                uint32_t pcn = 0;
                int nbn = 0;
                const int gotn = next_block(pcn, nbn);
                const int res = block_step<RES>(m, lds, hbase, nbk, pcl, L, tab, off0, z, a.blk_old);
                if (res == BLK_FALLBACK) {
#pragma unroll
                    for (int c = 0; c < FB; ++c) {
                        const int32_t j = c * 64 + static_cast<int32_t>(lane);
                        fstride[c] = j < z ? ld_w(&tab[j].stride) : 0;
                        fcode[c] = j < z ? ld_w(&tab[j].code) : 0xFFFFFFFFu;
                    }
                    for (int i = 0; i < nbk; ++i) {
                        ++r;
                        cur.prepare(m, lds, bcast(pcl, i), L, fstride, fcode);
                        uint32_t total, flags;
                        sweep_step<FB, RES>(m, lds, cur, fstride, fcode, L, dcap, total, flags);
                        if (flags == NZ_FLAGS) {
                            status = NZ_ST_DONE;
                            nstar = r;
                            mass = static_cast<int32_t>(total);
                            done = true;
                            break;
                        }
                    }
                    if (done) break;
                } else {
                    r += nbk;
                }
                got = gotn;
                pcl = pcn;
                nbk = nbn;
            }
            if (!done && got < 0) status = NZ_ST_BUCKET;
        } else {
        load_offsets();
        // The band in (key, site) order; the occupancy words of the next site are
        // loaded while the current one is processed.  Only the current site can
        // change them in between, so they are patched with its bit afterwards.
        BandCursor bc;
        bc.init(reinterpret_cast<const uint32_t *>(a.ws + d.off_counts),
                reinterpret_cast<const uint32_t *>(a.ws + d.off_sites), cap, nb);
        SiteStep<NCH, PER> cur, nxt;
        uint32_t pc = 0;
        int got = bc.next(pc, lane);
        if (got < 0) status = NZ_ST_BUCKET;
        if constexpr (kLookahead<NCH>) {
            if (got == 1) cur.prepare(m, lds, pc, L, ostride, ocode);
            while (got == 1) {
                ++r;
                uint32_t pcn = 0;
                const int gotn = bc.next(pcn, lane);
                if (gotn == 1) nxt.prepare(m, lds, pcn, L, ostride, ocode);
                uint32_t total, flags;
                sweep_step<NCH, RES>(m, lds, cur, ostride, ocode, L, dcap, total, flags);
                if (finished(total, flags)) break;
                if (gotn != 1) {
                    if (gotn < 0) status = NZ_ST_BUCKET;
                    break;
                }
                nxt.patch(cur.s, ostride, ocode, L);
                cur = nxt;
            }
        } else {
            while (got == 1) {
                ++r;
                cur.prepare(m, lds, pc, L, ostride, ocode);
                uint32_t total, flags;
                sweep_step<NCH, RES>(m, lds, cur, ostride, ocode, L, dcap, total, flags);
                if (finished(total, flags)) break;
                got = bc.next(pc, lane);
                if (got < 0) status = NZ_ST_BUCKET;
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

// ---------------------------------------------------------------------------
// Periodic boundaries: n* is the first addition after which a cluster wraps
// around axis 0 (Newman & Ziff 2001, Sec. III).
//
// Every site's entry is one 64-bit word: the low half is the parent word of the
// free-boundary sweep (a parent index, or a root word), the high half the x0
// displacement of the site from its parent in the unwrapped lattice (0 at a
// root).  A site's displacement from its root is the sum along its path.  Every
// write stores an (ancestor, displacement to it) pair in one 64-bit store, so
// any entry a lane or thread reads, however stale, is consistent.  An edge
// t = s + d inside one cluster closes a loop, and the loop winds around axis 0
// exactly when the displacements of s and t from their common root differ by
// anything but d0; the cluster then wraps and takes both border flags, the
// state the spanning test looks for.

__device__ __forceinline__ uint64_t wword(uint32_t par, int32_t dx)
{
    return (static_cast<uint64_t>(static_cast<uint32_t>(dx)) << 32) | par;
}
__device__ __forceinline__ int32_t wpar(uint64_t e) { return static_cast<int32_t>(static_cast<uint32_t>(e)); }
__device__ __forceinline__ int32_t wdx(uint64_t e) { return static_cast<int32_t>(e >> 32); }

// x0 component of an offset: the axis-0 field of its code has bit d0 + 2 set.
__device__ __forceinline__ int32_t code_d0(uint32_t code) { return __builtin_ctz(code | 32u) - 2; }

// Prefill phase: a root points to itself with displacement 0.  Root of x and
// the displacement of x from it; path splitting (each entry on the way skips to
// its grandparent, displacements added).
__device__ __forceinline__ int32_t ccw_find(uint64_t *pw, int32_t x, int32_t &disp)
{
    uint64_t e = ld_w(&pw[x]);
    int32_t D = 0;
    while (wpar(e) != x) {
        const int32_t p = wpar(e);
        const uint64_t g = ld_w(&pw[p]);
        if (wpar(g) != p) st_w(&pw[x], wword(static_cast<uint32_t>(wpar(g)), wdx(e) + wdx(g)));
        D += wdx(e);
        x = p;
        e = g;
    }
    disp = D;
    return x;
}

// Hook with displacements: as the free-boundary hook (CAS links the larger root
// below the smaller), the hooked root taking its displacement from the smaller
// one through the edge.  An edge whose ends already share a root is checked
// instead; a winding loop means the prefilled state already wraps, and the
// sample backs off.
__global__ __launch_bounds__(256) void nz_hookw_kernel(const NzSample *__restrict__ desc, const int32_t *__restrict__ list,
                                                       int32_t nlist, int32_t bx, const NzOffset *__restrict__ tabs,
                                                       uint8_t *__restrict__ ws, NzState *__restrict__ state)
{
    int32_t y, x;
    if (!xcd_slot(nlist, bx, y, x)) return;
    const int sid = list[y];
    const NzSample &d = desc[sid];
    const int32_t n0 = state[sid].n0;
    if (n0 > d.prefix_cap || !d.wrap) return;
    const int32_t L = d.L;
    const int32_t zh = d.z >> 1;
    const uint64_t magic = d.magic;
    uint64_t *pw = reinterpret_cast<uint64_t *>(ws + d.off_par);
    const uint32_t *occ = reinterpret_cast<const uint32_t *>(ws + d.off_occ);
    const uint32_t *prefix = reinterpret_cast<const uint32_t *>(ws + d.off_prefix);
    const NzOffset *tab = tabs + d.tab;
    bool wraps = false;
    for (int32_t i = x * 256 + static_cast<int32_t>(threadIdx.x); i < n0; i += bx * 256) {
        const int32_t s = static_cast<int32_t>(prefix[i]);
        const uint32_t pc = pack_coords(static_cast<uint32_t>(s), static_cast<uint32_t>(L), magic);
        const uint32_t A = allowed_axis(pc & 63, L) | (allowed_axis((pc >> 6) & 63, L) << 5) |
                           (allowed_axis((pc >> 12) & 63, L) << 10) | (allowed_axis((pc >> 18) & 63, L) << 15) |
                           (allowed_axis(pc >> 24, L) << 20);
        int32_t u = -1, Du = 0;   // a root (or ancestor) of s and the displacement of s from it
        for (int32_t k0 = 0; k0 < zh; k0 += HOOK_UNROLL) {
            int32_t t[HOOK_UNROLL], d0[HOOK_UNROLL];
            uint32_t w[HOOK_UNROLL];
#pragma unroll
            for (int q = 0; q < HOOK_UNROLL; ++q) {
                NzOffset o;
                o.stride = 0;
                o.code = 0xFFFFFFFFu;
                if (k0 + q < zh) o = tab[k0 + q];
                const uint32_t out = o.code & ~A;
                const bool ok = (o.code & ~kCodeBits) == 0u;   // every real offset, wrapped
                t[q] = s + o.stride + (out ? wrap_fix(out, L) : 0);
                d0[q] = code_d0(o.code);
                w[q] = ok ? occ[static_cast<uint32_t>(t[q]) >> 5] : 0u;
            }
#pragma unroll
            for (int q = 0; q < HOOK_UNROLL; ++q) {
                if (!((w[q] >> (t[q] & 31)) & 1u)) continue;
                if (u < 0) u = ccw_find(pw, s, Du);
                int32_t Dv;
                int32_t v = ccw_find(pw, t[q], Dv);
                for (;;) {
                    if (u == v) {
                        if (Du + d0[q] != Dv) wraps = true;
                        break;
                    }
                    const int32_t hi = max(u, v), lo = min(u, v);
                    // x0(u) = x0(s) - Du and x0(v) = x0(s) + d0 - Dv
                    const int32_t dx = hi == u ? Dv - Du - d0[q] : Du + d0[q] - Dv;
                    uint64_t expected = wword(static_cast<uint32_t>(hi), 0);
                    if (__hip_atomic_compare_exchange_strong(&pw[hi], &expected, wword(static_cast<uint32_t>(lo), dx),
                                                             __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        if (hi == u) {
                            u = lo;
                            Du += dx;
                        }
                        break;
                    }
                    // hi is no longer a root: go on from the entry the CAS returned
                    int32_t Dp;
                    if (u == hi) {
                        u = ccw_find(pw, wpar(expected), Dp);
                        Du += wdx(expected) + Dp;
                    } else {
                        u = ccw_find(pw, u, Dp);
                        Du += Dp;
                    }
                    if (v == hi) {
                        v = ccw_find(pw, wpar(expected), Dp);
                        Dv += wdx(expected) + Dp;
                    } else {
                        v = ccw_find(pw, v, Dp);
                        Dv += Dp;
                    }
                }
            }
        }
    }
    if (wraps) state[sid].status = NZ_ST_BACKOFF;
}

// Compress with displacements: every member holds (root, displacement from the
// root), every root its root word (size 1, no border flags).  Walks are
// read-only and each thread writes only its own entry, as in the
// free-boundary compress.
__global__ __launch_bounds__(256) void nz_compressw_kernel(const NzSample *__restrict__ desc, const int32_t *__restrict__ list,
                                                           int32_t nlist, int32_t bx, uint8_t *__restrict__ ws,
                                                           NzState *__restrict__ state)
{
    int32_t y, x;
    if (!xcd_slot(nlist, bx, y, x)) return;
    const int sid = list[y];
    const NzSample &d = desc[sid];
    const int32_t n0 = state[sid].n0;
    if (n0 > d.prefix_cap || !d.wrap) return;
    uint64_t *pw = reinterpret_cast<uint64_t *>(ws + d.off_par);
    const uint32_t *prefix = reinterpret_cast<const uint32_t *>(ws + d.off_prefix);
    for (int32_t k = x * 256 + static_cast<int32_t>(threadIdx.x); k < n0; k += bx * 256) {
        const int32_t s = static_cast<int32_t>(prefix[k]);
        int32_t r = s, D = 0;
        uint64_t e = ld_w(&pw[r]);
        while (wpar(e) >= 0 && wpar(e) != r) {
            D += wdx(e);
            r = wpar(e);
            e = ld_w(&pw[r]);
        }
        st_w(&pw[s], r == s ? wword(NZ_ROOT | 1u, 0) : wword(static_cast<uint32_t>(r), D));
    }
}

// Sizes of the prefilled clusters: members add themselves to the low half of
// their root's entry.
__global__ __launch_bounds__(256) void nz_accumw_kernel(const NzSample *__restrict__ desc, const int32_t *__restrict__ list,
                                                        int32_t nlist, int32_t bx, uint8_t *__restrict__ ws,
                                                        NzState *__restrict__ state)
{
    int32_t y, x;
    if (!xcd_slot(nlist, bx, y, x)) return;
    const int sid = list[y];
    const NzSample &d = desc[sid];
    if (!d.wrap) return;
    const int32_t n0 = state[sid].n0;
    if (n0 > d.prefix_cap) {
        if (x == 0 && threadIdx.x == 0) state[sid].status = NZ_ST_PREFIX;
        return;
    }
    uint64_t *pw = reinterpret_cast<uint64_t *>(ws + d.off_par);
    const uint32_t *prefix = reinterpret_cast<const uint32_t *>(ws + d.off_prefix);
    for (int32_t k = x * 256 + static_cast<int32_t>(threadIdx.x); k < n0; k += bx * 256) {
        const int32_t s = static_cast<int32_t>(prefix[k]);
        const int32_t r = wpar(pw[s]);
        if (r >= 0) atomicAdd(reinterpret_cast<uint32_t *>(&pw[r]), 1u);   // low half: the root word
    }
}

// Sweep phase: root of x, its root word and the displacement of x from it; path
// halving with displacements added.
__device__ __forceinline__ void wrap_find(uint64_t *pw, int32_t x, int32_t &root, uint32_t &word, int32_t &disp)
{
    uint64_t e = ld_w(&pw[x]);
    int32_t D = 0;
    while (wpar(e) >= 0) {
        const int32_t p = wpar(e);
        const uint64_t g = ld_w(&pw[p]);
        if (wpar(g) < 0) {
            D += wdx(e);
            x = p;
            e = g;
            break;
        }
        const uint64_t h = wword(static_cast<uint32_t>(wpar(g)), wdx(e) + wdx(g));
        st_w(&pw[x], h);
        D += wdx(h);
        x = wpar(g);
        e = ld_w(&pw[x]);
    }
    root = x;
    word = static_cast<uint32_t>(wpar(e));
    disp = D;
}

// Merge the D distinct roots held by lanes 0..D-1 into the largest (ties: the
// smaller index).  lq is x0(new site) - x0(lane's root); each attached root
// takes its displacement from the survivor.  Returns the survivor and, through
// the references, the total size, the flags and the survivor's lq.
__device__ __forceinline__ int32_t wrap_merge(uint64_t *pw, int D, int32_t lroot, uint32_t lword, int32_t lq,
                                              uint32_t wrapfl, uint32_t &total, uint32_t &flags, int32_t &qbest)
{
    const uint32_t lane = lane_id();
    int32_t best = bcast(lroot, 0);
    uint32_t bestsz = bcast(lword, 0) & NZ_SIZE;
    int bl = 0;
    total = 0;
    flags = wrapfl;
    for (int l = 0; l < D; ++l) {
        const int32_t r = bcast(lroot, l);
        const uint32_t w = bcast(lword, l);
        const uint32_t sz = w & NZ_SIZE;
        total += sz;
        flags |= w & NZ_FLAGS;
        if (sz > bestsz || (sz == bestsz && r < best)) {
            best = r;
            bestsz = sz;
            bl = l;
        }
    }
    qbest = bcast(lq, bl);
    // x0(root) - x0(best) = (x0(site) - lq) - (x0(site) - qbest)
    if (static_cast<int>(lane) < D && lroot != best) st_w(&pw[lroot], wword(static_cast<uint32_t>(best), qbest - lq));
    st_w(&pw[best], wword(NZ_ROOT | flags | total, 0));   // every lane, same value
    return best;
}

// One addition under periodic boundaries: as the free-boundary step, with the
// new site's displacement from each neighbouring root carried along and
// compared whenever two neighbours share a root.
template <int NCH>
__device__ __forceinline__ void wrap_step(uint32_t *occ, uint64_t *pw, const SiteStep<NCH, true> &cur, const int32_t (&od0)[NCH],
                                          const int32_t (&ostride)[NCH], const uint32_t (&ocode)[NCH], int32_t L,
                                          int dcap, uint32_t &total, uint32_t &flags)
{
    const uint32_t lane = lane_id();
    const int32_t s = cur.s;
    st_w(&occ[static_cast<uint32_t>(s) >> 5], cur.own | (1u << (s & 31)));

    int32_t lroot = s, lq = 0;
    uint32_t lword = NZ_ROOT | 1u;
    uint32_t wrapfl = 0;
    int D = 1;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int32_t t = cur.nbr(c, ostride, ocode, L);
        const bool o = (cur.word[c] >> (t & 31)) & 1u;   // the word is 0 outside the lattice
        uint64_t mk = __ballot(o);
        if (!mk) continue;
        int32_t root = 0, disp = 0;
        uint32_t rw = 0;
        if (o) wrap_find(pw, t, root, rw, disp);
        // t = s + d: x0(s) - x0(root) = disp - d0
        const int32_t q = disp - od0[c];
        bool stale = false;   // a flush since these finds may have linked their roots
        while (mk) {
            const int l = __builtin_ctzll(mk);
            mk &= mk - 1;
            int32_t rr = bcast(root, l);
            uint32_t rrw = bcast(rw, l);
            int32_t qq = bcast(q, l);
            if (stale) {
                int32_t extra;
                wrap_find(pw, rr, rr, rrw, extra);
                qq += extra;
            }
            const uint64_t hit = __ballot(static_cast<int>(lane) < D && lroot == rr);
            if (hit) {
                if (bcast(lq, __builtin_ctzll(hit)) != qq) wrapfl = NZ_FLAGS;
                continue;
            }
            if (D == dcap) {
                uint32_t tot, flg;
                int32_t qb;
                const int32_t w = wrap_merge(pw, D, lroot, lword, lq, wrapfl, tot, flg, qb);
                lroot = lane == 0 ? w : lroot;
                lword = lane == 0 ? (NZ_ROOT | flg | tot) : lword;
                lq = lane == 0 ? qb : lq;
                D = 1;
                stale = true;
            }
            lroot = static_cast<int>(lane) == D ? rr : lroot;
            lword = static_cast<int>(lane) == D ? rrw : lword;
            lq = static_cast<int>(lane) == D ? qq : lq;
            ++D;
        }
    }
    int32_t qb;
    wrap_merge(pw, D, lroot, lword, lq, wrapfl, total, flags, qb);
}

// Persistent first-wrap sweep: one wave per sample, one site per step, state
// in HBM (the entries are twice as wide as in the free-boundary sweep).
template <int NCH>
__global__ __launch_bounds__(256) void nz_wrap_sweep_kernel(NzSweepArgs a, SweepOut out)
{
    __shared__ int32_t claim[4];
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x >> 6;
    for (;;) {
        if (lane == 0) claim[wave] = atomicAdd(a.qhead, 1);
        __builtin_amdgcn_wave_barrier();
        const int qi = __builtin_amdgcn_readfirstlane(ld_w(&claim[wave]));
        __builtin_amdgcn_wave_barrier();
        if (qi >= a.nqueue) break;
        const int sid = a.queue[qi];
        if (a.state[sid].status != NZ_ST_PENDING) continue;
        const NzSample &d = a.desc[sid];
        const int32_t L = d.L;
        const int32_t z = d.z;
        SweepMem<RES_HBM> m;
        m.occ_g = reinterpret_cast<uint32_t *>(a.ws + d.off_occ);
        m.par_g = nullptr;   // the occupancy side only; entries go through pw
        m.parc_g = nullptr;
        m.lbase = 0;
        m.occ_words = 0;
        m.sshift = 0;
        m.sum_on = false;   // no summary: every check reads the bitset
        uint64_t *pw = reinterpret_cast<uint64_t *>(a.ws + d.off_par);
        const NzOffset *tab = a.tabs + d.tab;
        int32_t ostride[NCH], od0[NCH];
        uint32_t ocode[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int32_t j = c * 64 + static_cast<int32_t>(lane);
            const NzOffset o = j < z ? tab[j] : NzOffset{0, 0xFFFFFFFFu};
            ostride[c] = o.stride;
            ocode[c] = o.code;
            od0[c] = code_d0(o.code);
        }
        int32_t r = a.state[sid].n0;
        int32_t status = NZ_ST_BAND;
        int32_t nstar = 0, mass = 0;
        BandCursor bc;
        bc.init(reinterpret_cast<const uint32_t *>(a.ws + d.off_counts),
                reinterpret_cast<const uint32_t *>(a.ws + d.off_sites), static_cast<uint32_t>(d.cap), d.nb);
        SiteStep<NCH, true> cur;
        uint32_t pc = 0;
        int got = bc.next(pc, lane);
        while (got == 1) {
            ++r;
            cur.prepare(m, nullptr, pc, L, ostride, ocode);
            uint32_t total, flags;
            wrap_step<NCH>(m.occ_g, pw, cur, od0, ostride, ocode, L, a.dcap, total, flags);
            if (flags == NZ_FLAGS) {
                status = NZ_ST_DONE;
                nstar = r;
                mass = static_cast<int32_t>(total);
                break;
            }
            got = bc.next(pc, lane);
        }
        if (got < 0) status = NZ_ST_BUCKET;
        if (status == NZ_ST_BAND && d.full) {
            status = NZ_ST_DONE;   // every site occupied and nothing wraps
            nstar = 0;
            mass = 0;
        }
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
                       NzState *state, int32_t max_grid, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int32_t bps = (N + KEYS_SITES_PER_BLOCK - 1) / KEYS_SITES_PER_BLOCK;
    const int64_t blocks = static_cast<int64_t>(bps) * count;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    const int64_t grid = max_grid > 0 ? std::min<int64_t>(blocks, max_grid) : blocks;
    hipLaunchKernelGGL(nz_keys_kernel, dim3(static_cast<uint32_t>(grid)), dim3(KEYS_THREADS), 0, st, desc, list, first,
                       bps, static_cast<int32_t>(blocks), ws, state);
    return hipGetLastError();
}

int32_t keys_sites_per_block() { return KEYS_SITES_PER_BLOCK; }

int32_t keys_resident_wgs()
{
    // one kernel, one architecture: the answer is fixed for the process
    static const int32_t wgs = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, nz_keys_kernel, KEYS_THREADS, 0) != hipSuccess || n < 1) n = 1;
        return static_cast<int32_t>(n);
    }();
    return wgs;
}

hipError_t launch_sort(const NzSample *desc, int32_t nsamp, int32_t max_nb, int32_t max_cap, uint8_t *ws,
                       hipStream_t st)
{
    if (nsamp <= 0 || max_nb <= 0) return hipSuccess;
    uint32_t P = 2;
    while (P < static_cast<uint32_t>(max_cap)) P <<= 1;
    const int64_t items = static_cast<int64_t>(nsamp) * max_nb;
    if (items > 0x7FFFFFFFll) return hipErrorInvalidValue;   // the waves step through items in 32 bits
    // one wave per bucket; as many waves per workgroup as 64 KB of LDS holds
    const size_t per_wave = static_cast<size_t>(P) * (sizeof(uint64_t) + sizeof(uint32_t));
    const int waves = static_cast<int>(std::max<size_t>(1, std::min<size_t>(SORT_THREADS / 64, 65536 / per_wave)));
    const size_t lds = per_wave * static_cast<size_t>(waves);
    auto k = nz_sort_kernel;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    const int64_t blocks = (items + waves - 1) / waves;
    const uint32_t grid = static_cast<uint32_t>(blocks < 65536 * 4 ? blocks : 65536 * 4);
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * waves), lds, st, desc, nsamp, max_nb, P, ws);
    return hipGetLastError();
}

hipError_t launch_prefill(const NzSample *desc, const int32_t *list, int32_t nlist, int32_t bx_hook, int32_t bx_site,
                          const NzOffset *tabs, uint8_t *ws, NzState *state, bool smax, bool wrap, bool periodic,
                          hipStream_t st, hipEvent_t *ev)
{
    if (nlist <= 0) return hipSuccess;
    auto mark = [&](int k) {
        if (ev) (void)hipEventRecord(ev[k], st);
    };
    mark(0);
    const uint32_t slots8 = static_cast<uint32_t>((nlist + 7) / 8) * 8u;
    if (wrap) {
        hipLaunchKernelGGL(nz_hookw_kernel, dim3(static_cast<uint32_t>(bx_hook) * slots8), dim3(256), 0, st, desc, list,
                           nlist, bx_hook, tabs, ws, state);
        hipLaunchKernelGGL(nz_compressw_kernel, dim3(static_cast<uint32_t>(bx_site) * slots8), dim3(256), 0, st, desc, list,
                           nlist, bx_site, ws, state);
        hipLaunchKernelGGL(nz_accumw_kernel, dim3(static_cast<uint32_t>(bx_site) * slots8), dim3(256), 0, st, desc, list,
                           nlist, bx_site, ws, state);
        mark(1);
        mark(2);
        mark(3);
        mark(4);
        return hipGetLastError();
    }
    if (periodic)
        hipLaunchKernelGGL(nz_hook_kernel<true>, dim3(static_cast<uint32_t>(bx_hook) * slots8), dim3(256), 0, st, desc, list,
                           nlist, bx_hook, tabs, ws, state);
    else
        hipLaunchKernelGGL(nz_hook_kernel<false>, dim3(static_cast<uint32_t>(bx_hook) * slots8), dim3(256), 0, st, desc,
                           list, nlist, bx_hook, tabs, ws, state);
    mark(1);
    hipLaunchKernelGGL(nz_compress_kernel, dim3(static_cast<uint32_t>(bx_site) * slots8), dim3(256), 0, st, desc, list,
                       nlist, bx_site, ws, state);
    mark(2);
    hipLaunchKernelGGL(nz_accum_kernel, dim3(static_cast<uint32_t>(bx_site) * slots8), dim3(256), 0, st, desc, list, nlist,
                       bx_site, ws, state);
    mark(3);
    mark(4);   // (the lattice entries are written by the size pass)
    if (smax)
        hipLaunchKernelGGL(nz_rootmax_kernel, dim3(static_cast<uint32_t>(bx_site) * slots8), dim3(256), 0, st, desc, list,
                           nlist, bx_site, ws, state);
    return hipGetLastError();
}

hipError_t launch_winsum(const NzSample *desc, const NzState *state, int32_t nsamp, int32_t w, const uint8_t *ws,
                         uint64_t *out, hipStream_t st)
{
    if (nsamp <= 0 || w <= 0) return hipSuccess;
    const int32_t blocks = (w + 255) / 256;
    const uint32_t grid = static_cast<uint32_t>(blocks < 4096 ? blocks : 4096);
    hipLaunchKernelGGL(nz_winsum_kernel, dim3(grid), dim3(256), 0, st, desc, state, nsamp, w, ws, out);
    return hipGetLastError();
}

template <int NCH, int RES, bool BLOCK, bool PER, int FB = NCH>
static hipError_t launch_sweep_t(const NzSweepArgs &a, const SweepOut &o, int grid, int wg_waves, size_t lds,
                                 hipStream_t st)
{
    auto k = nz_sweep_kernel<NCH, RES, BLOCK, FB, PER>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * wg_waves), lds, st, a, o);
    return hipGetLastError();
}

template <int RES, bool BLOCK, bool PER = false>
static hipError_t launch_sweep_r(int nch, bool wide_block, const NzSweepArgs &a, const SweepOut &o, int grid,
                                 int wg_waves, size_t lds, hipStream_t st)
{
    switch (nch) {
    case 1: return launch_sweep_t<1, RES, BLOCK, PER>(a, o, grid, wg_waves, lds, st);
    case 2: return launch_sweep_t<2, RES, BLOCK, PER>(a, o, grid, wg_waves, lds, st);
    case 4: return launch_sweep_t<4, RES, BLOCK, PER>(a, o, grid, wg_waves, lds, st);
    case 8: return launch_sweep_t<8, RES, BLOCK, PER>(a, o, grid, wg_waves, lds, st);
    case 14:
        if constexpr (BLOCK) {
            if (!wide_block) return launch_sweep_t<14, RES, BLOCK, PER, 8>(a, o, grid, wg_waves, lds, st);
        }
        return launch_sweep_t<14, RES, BLOCK, PER>(a, o, grid, wg_waves, lds, st);
    default: return hipErrorInvalidValue;
    }
}

uint32_t block_lds_words() { return BLK_LDS_WORDS; }

hipError_t launch_wrap_sweep(int nch, const NzSweepArgs &a, int32_t *nstar, int32_t *mass, const int32_t *out_index,
                             int grid, hipStream_t st)
{
    SweepOut o{nstar, mass, out_index};
    switch (nch) {
    case 1: hipLaunchKernelGGL(nz_wrap_sweep_kernel<1>, dim3(grid), dim3(256), 0, st, a, o); break;
    case 2: hipLaunchKernelGGL(nz_wrap_sweep_kernel<2>, dim3(grid), dim3(256), 0, st, a, o); break;
    case 4: hipLaunchKernelGGL(nz_wrap_sweep_kernel<4>, dim3(grid), dim3(256), 0, st, a, o); break;
    case 8: hipLaunchKernelGGL(nz_wrap_sweep_kernel<8>, dim3(grid), dim3(256), 0, st, a, o); break;
    case 14: hipLaunchKernelGGL(nz_wrap_sweep_kernel<14>, dim3(grid), dim3(256), 0, st, a, o); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sweep(int nch, bool wide_block, int residency, bool block, bool periodic, const NzSweepArgs &a,
                        int32_t *nstar, int32_t *mass, const int32_t *out_index, int grid, int wg_waves, hipStream_t st)
{
    SweepOut o{nstar, mass, out_index};
    const size_t lds = static_cast<size_t>(a.lds_words) * 4u * static_cast<size_t>(wg_waves);
    if (periodic) {
        if (block) return hipErrorInvalidValue;
        switch (residency) {
        case RES_HBM: return launch_sweep_r<RES_HBM, false, true>(nch, false, a, o, grid, wg_waves, lds, st);
        case RES_OCC: return launch_sweep_r<RES_OCC, false, true>(nch, false, a, o, grid, wg_waves, lds, st);
        case RES_ALL: return launch_sweep_r<RES_ALL, false, true>(nch, false, a, o, grid, wg_waves, lds, st);
        default: return hipErrorInvalidValue;
        }
    }
    if (block) {
        switch (residency) {
        case RES_HBM: return launch_sweep_r<RES_HBM, true>(nch, wide_block, a, o, grid, wg_waves, lds, st);
        case RES_OCC: return launch_sweep_r<RES_OCC, true>(nch, wide_block, a, o, grid, wg_waves, lds, st);
        case RES_ALL: return launch_sweep_r<RES_ALL, true>(nch, wide_block, a, o, grid, wg_waves, lds, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (residency) {
    case RES_HBM: return launch_sweep_r<RES_HBM, false>(nch, wide_block, a, o, grid, wg_waves, lds, st);
    case RES_OCC: return launch_sweep_r<RES_OCC, false>(nch, wide_block, a, o, grid, wg_waves, lds, st);
    case RES_ALL: return launch_sweep_r<RES_ALL, false>(nch, wide_block, a, o, grid, wg_waves, lds, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nz
