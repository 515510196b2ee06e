// nz_internal.h -- records shared by the host planner (nz_api.cpp) and the
// HIP kernels (nz_kernels.hip).  Not part of the public ABI.
#pragma once
#include <stdint.h>

// Root word of the union-find (one int32 per site, Sec. II.B construction):
//   bit 31 set      -> the site is a cluster root; bits 0..28 hold the cluster
//                      size, bit 30 "a member has x0 = 0", bit 29 "a member has
//                      x0 = L-1";
//   bit 31 clear    -> the value is the index of the site's parent.
// Sizes need 29 bits, hence L <= 55 (55^5 < 2^29).
#define NZ_ROOT 0x80000000u
#define NZ_FLO 0x40000000u
#define NZ_FHI 0x20000000u
#define NZ_FLAGS (NZ_FLO | NZ_FHI)
#define NZ_SIZE 0x1FFFFFFFu

// Per-sample status written by the kernels.
enum {
    NZ_ST_PENDING = 0,
    NZ_ST_DONE = 1,       // n*, mass final
    NZ_ST_BAND = 2,       // the key band ran out before the sample spanned: redo wider
    NZ_ST_BUCKET = 3,     // a sort bucket overflowed before the sample spanned: redo finer
    NZ_ST_BACKOFF = 4,    // the prefilled state already spans: redo with a smaller n0
    NZ_ST_PREFIX = 5,     // the prefill list overflowed: redo with a larger list
};

// One neighbour offset of a (zone mask, L) table.  stride is the change of the
// linear site index; code has, for each axis j, bit (5*j + d_j + 2) set, so the
// offset stays inside the lattice iff (code & ~allowed(x)) == 0, where
// allowed(x) has bit (5*j + d + 2) set iff 0 <= x_j + d < L.
struct NzOffset {
    int32_t stride;
    uint32_t code;
};

// Per-sample descriptor (one per sample of a chunk), built by the host.
struct NzSample {
    uint64_t seed;
    uint64_t sample;
    uint64_t T0;          // keys below T0 are occupied before the sweep (0: plain)
    uint64_t off_par;     // byte offsets into the workspace
    uint64_t off_occ;
    uint64_t off_keys;
    uint64_t off_sites;
    uint64_t off_counts;
    uint64_t off_prefix;  // prefilled sites in list order (site order within each key block)
    uint64_t off_parc;    // parents of the list entries during the bulk labelling
    uint64_t off_wpos;    // per bitset word: list position of its first prefilled site
    int32_t L;
    int32_t N;
    int32_t nb;           // buckets of the key band [T0, T0 + nb << shift)
    int32_t cap;          // capacity of each bucket (entries)
    int32_t shift;        // log2 of the bucket width in key units
    int32_t full;         // the band reaches 2^64 (exhaustion then means "never spans")
    int32_t tab;          // first entry of this sample's offset table
    int32_t z;            // number of offsets
    int32_t prefix_cap;   // capacity of the prefill site list
    int32_t smax_mode;    // 1: track the largest cluster over [win_lo, win_hi) instead of stopping at n*
    uint64_t magic;       // ceil(2^64 / L) for exact division of site indices by L
    uint64_t off_win;     // smax mode: S_max(n) for n in [win_lo, win_hi), uint32 each
    int32_t win_lo;
    int32_t win_hi;
    int32_t periodic;     // 1: coordinates wrap mod L (L >= 5); no borders, so no border flags
    int32_t wrap;         // 1: periodic first-wrap sweep; entries of off_par are 64-bit
                          //    (low half the parent word, high half the x0 displacement
                          //    from the parent)
    uint64_t off_sum;     // bitset summary: bit k set unless words k << sum_shift .. are all zero
    int32_t sum_shift;
    int32_t sum_words;    // 32-bit summary words (0: no summary)
};

// Per-sample result/state record written by the kernels.
struct NzState {
    int32_t status;
    int32_t nstar;
    int32_t mass;
    int32_t n0;           // sites occupied by the prefill (count of keys < T0)
    int32_t smax;         // smax mode: largest cluster of the prefilled state
};

// Launch parameters of the sweep (one persistent launch per chunk).
struct NzSweepArgs {
    const NzSample *desc;
    const int32_t *queue;     // sample indices, longest first
    int32_t nqueue;
    int32_t *qhead;           // work counter, zero at launch
    const NzOffset *tabs;
    uint8_t *ws;
    NzState *state;
    uint32_t lds_words;       // 32-bit LDS words per wave (LDS residencies)
    int32_t dcap;             // distinct roots held per step before an early merge (2..64)
    int32_t blk_old;          // block sweep: earlier roots one block may touch (0..256)
    int32_t blk_zmax;         // block sweep for samples with z <= blk_zmax, one site per step above
    int32_t use_sum;          // 1: HBM-resident samples check the bitset summary before occupancy loads
};
