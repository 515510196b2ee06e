// nz_api.cpp -- the C ABI of libnz (include/nz.h): argument checking, the
// neighbourhood tables, the per-sample plan (key band, buckets, prefill),
// workspace layout, chunked launches on one stream and the redo loop for the
// rare samples whose band or bucket ran short or whose prefill already spans.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/nz.h"
#include "nz_internal.h"
#include "nz_launch.h"

#define NZ_API extern "C" __attribute__((visibility("default")))

namespace {

thread_local std::string g_err = "no error";
thread_local int64_t g_stats[6] = {0, 0, 0, 0, 0, 0};
thread_local bool g_timing = false;
thread_local double g_ms[6] = {0, 0, 0, 0, 0, 0};
// per job of the last batch (caller's job order): sequential additions and
// sites occupied by the bulk prefill, summed over the final runs of its samples
thread_local std::vector<int64_t> g_job_serial, g_job_pre;
// bulk-labelling kernels of the last batch: milliseconds in hook, compress and
// the size pass (summed over dispatches), 0 (no separate expand pass) and the
// number of dispatches
thread_local double g_cc_ms[5] = {0, 0, 0, 0, 0};

// Events around each kernel of the bulk labelling; a chunk launches it up to
// three times (the first pass and two in-chunk backoffs).
struct PrefillEvents {
    hipEvent_t ev[3][5] = {};
    int used = 0;
    bool ok = false;
    PrefillEvents()
    {
        ok = true;
        for (auto &row : ev)
            for (auto &e : row) ok = ok && hipEventCreate(&e) == hipSuccess;
    }
    ~PrefillEvents()
    {
        for (auto &row : ev)
            for (auto &e : row)
                if (e) (void)hipEventDestroy(e);
    }
};

// Events bracketing the phases of one chunk (keys, prefill, sort, sweep).
struct PhaseEvents {
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool ok = false;
    PhaseEvents()
    {
        ok = true;
        for (auto &e : ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    }
    ~PhaseEvents()
    {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(NZ_EDEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),   \
                        __FILE__, __LINE__);                                                 \
    } while (0)

int64_t pow5(int64_t L) { return L * L * L * L * L; }

// ---------------------------------------------------------------------------
// Neighbourhoods (Sec. II.A.2, Table I): zone k is the shell |d|^2 = k of Z^5,
// k = 1..7.  Every shell vector has |d_j| <= 2.  The table lists first the
// vectors whose last non-zero coordinate is negative and then their negations
// in the same order, so its first half holds one vector of every +-d pair.

std::vector<std::array<int, 5>> enumerate_zone_vectors(uint32_t mask)
{
    std::vector<std::array<int, 5>> neg;
    for (int k = 1; k <= 7; ++k) {
        if (!(mask >> (k - 1) & 1u)) continue;
        for (int v = 0; v < 3125; ++v) {
            std::array<int, 5> d;
            int r2 = 0, rem = v;
            for (int j = 0; j < 5; ++j) {
                d[j] = rem % 5 - 2;
                rem /= 5;
                r2 += d[j] * d[j];
            }
            if (r2 != k) continue;
            int last = 0;
            for (int j = 4; j >= 0; --j)
                if (d[j] != 0) {
                    last = d[j];
                    break;
                }
            if (last < 0) neg.push_back(d);
        }
    }
    std::vector<std::array<int, 5>> all = neg;
    for (const auto &d : neg) all.push_back({-d[0], -d[1], -d[2], -d[3], -d[4]});
    return all;
}

// The vectors of every mask 1..127, enumerated once per process (mask 0 and
// masks above 127 give the empty list).
const std::vector<std::array<int, 5>> &zone_vectors(uint32_t mask)
{
    static const std::array<std::vector<std::array<int, 5>>, 128> all = [] {
        std::array<std::vector<std::array<int, 5>>, 128> t;
        for (uint32_t m = 1; m < 128; ++m) t[m] = enumerate_zone_vectors(m);
        return t;
    }();
    return all[mask < 128 ? mask : 0];
}

// z(mask) for every mask, enumerated once.
int coordination(uint32_t mask)
{
    static const std::array<int, 128> z = [] {
        std::array<int, 128> t{};
        for (uint32_t m = 1; m < 128; ++m) t[m] = static_cast<int>(zone_vectors(m).size());
        return t;
    }();
    return mask >= 1 && mask <= 127 ? z[mask] : -1;
}

std::vector<NzOffset> build_table(uint32_t mask, int32_t L)
{
    std::vector<NzOffset> t;
    for (const auto &d : zone_vectors(mask)) {
        NzOffset o;
        int64_t stride = 0, p = 1;
        uint32_t code = 0;
        for (int j = 0; j < 5; ++j) {
            stride += d[j] * p;
            p *= L;
            code |= 1u << (5 * j + d[j] + 2);
        }
        o.stride = static_cast<int32_t>(stride);
        o.code = code;
        t.push_back(o);
    }
    return t;
}

// ---------------------------------------------------------------------------
// Device facts.

struct Device {
    int id = -1;
    int cus = 256;
    size_t lds_per_block = 65536;
    size_t lds_per_cu = 65536;
};

int device_info(Device &dev)
{
    int id = 0;
    HIP_TRY(hipGetDevice(&id));
    // one cache for the process (the two-group path queries from a second thread)
    static std::mutex lock;
    static std::map<int, Device> cache;
    {
        std::lock_guard<std::mutex> g(lock);
        auto it = cache.find(id);
        if (it != cache.end()) {
            dev = it->second;
            return NZ_OK;
        }
    }
    hipDeviceProp_t p;
    HIP_TRY(hipGetDeviceProperties(&p, id));
    dev.id = id;
    dev.cus = p.multiProcessorCount;
    dev.lds_per_block = p.sharedMemPerBlock;
    dev.lds_per_cu = p.maxSharedMemoryPerMultiProcessor ? p.maxSharedMemoryPerMultiProcessor : p.sharedMemPerBlock;
    int optin = 0;
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, id) == hipSuccess && optin > 0)
        dev.lds_per_block = std::max(dev.lds_per_block, static_cast<size_t>(optin));
    std::lock_guard<std::mutex> g(lock);
    cache[id] = dev;
    return NZ_OK;
}

// ---------------------------------------------------------------------------
// Per-sample plan.

constexpr int kMaxChunk = 16384;
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Threshold coefficient of p_c = c / (z + b) fitted over Table I (Sec. III.B:
// c ~ 1.553, b ~ 1.01); used only to size key bands and to order work.
double pc_prior(int z) { return 1.553 / (z + 1.01); }

// 32-bit words of a sample's bitset summary in the sweep's LDS slice
constexpr int64_t kSumWords = 1024;
// The sweep consults the summary (automatic choice) when its chunk has at least
// this many samples per CU: measured at L = 16..24, the skipped loads pay once
// several waves share a CU, while at about one wave per CU the extra LDS read
// before each load costs 5-20% of the sweep.
constexpr int32_t kSumSamplesPerCu = 2;

struct Plan {
    int32_t job;
    int64_t sample;      // Philox sample index
    int32_t out;         // index into the caller's output arrays
    int32_t L;
    uint32_t mask;
    int64_t n0;          // current prefill rank (0: plain)
    int64_t backoff;     // backoff step still available (0: next backoff goes to 0)
    int64_t band_hi;     // upper end of the key band in sites
    int32_t shift_adj;   // extra halvings of the bucket width
    int32_t prefix_mul;  // prefill list capacity multiplier
    double prio;
    int64_t win_lo, win_hi;   // smax mode: S_max(n) for n in [win_lo, win_hi) (win_hi = 0: off)
    bool wrap;           // periodic first-wrap sample (64-bit union-find entries)
    bool per;            // periodic coordinates (first-wrap or largest-cluster windows)
};

uint64_t rank_to_key(int64_t n, int64_t N)
{
    // floor(n / N * 2^64) for 0 <= n < N
    unsigned __int128 v = (static_cast<unsigned __int128>(static_cast<uint64_t>(n)) << 64) / static_cast<uint64_t>(N);
    return static_cast<uint64_t>(v);
}

// Prefill key threshold for rank n: rank_to_key rounded down to a multiple of
// 2^32, so that the keys kernel tests keys against it (and against the band's
// end, a whole number of buckets of at least 2^32 keys above it) by their high
// words.  The prefill is whatever lies below the threshold: n* and the mass
// never depend on it, and the rounding moves it by under N / 2^32 sites.
uint64_t prefill_key(int64_t n, int64_t N)
{
    // test hook: the unrounded threshold drives the keys kernel's 64-bit compares
    if (getenv("NZ_DEBUG_EXACT_T0")) return rank_to_key(n, N);
    const uint64_t t = rank_to_key(n, N) & ~0xFFFFFFFFull;
    return t != 0 ? t : rank_to_key(n, N);   // (n >= 1 and N < 2^32 keep it nonzero)
}

struct Sizes {
    uint64_t T0;
    int32_t nb, cap, shift, full, prefix_cap;
    // prefill ranks of the backoffs resolved inside the chunk: n0 - b, then
    // n0 - 3b (0: none planned), their key thresholds and band buckets
    int64_t n0b[2];
    uint64_t T0b[2];
    int32_t nbb[2];
    size_t par, occ, keys, sites, counts, prefix, parc, wpos, win, sum, total;
    int32_t sum_shift, sum_words;
};

Sizes plan_sizes(const Plan &p, int bucket_log2)
{
    Sizes s{};
    const int64_t N = pow5(p.L);
    s.T0 = p.n0 > 0 ? prefill_key(p.n0, N) : 0;
    int lgN = 0;
    while ((int64_t(1) << lgN) < N) ++lgN;
    int shift = 64 + bucket_log2 - lgN - p.shift_adj;
    shift = std::max(1, std::min(63, shift));
    s.shift = shift;
    s.full = p.band_hi >= N ? 1 : 0;
    const uint64_t Thi = s.full ? 0 : rank_to_key(std::max<int64_t>(p.band_hi, p.n0 + 1), N);
    // buckets of width 2^shift covering [T, Thi) (or [T, 2^64) for a full band)
    auto buckets = [&](uint64_t T) {
        const unsigned __int128 top = s.full ? (static_cast<unsigned __int128>(1) << 64) : Thi;
        const unsigned __int128 span = top > T ? top - T : 1;
        const unsigned __int128 w = static_cast<unsigned __int128>(1) << shift;
        return static_cast<int32_t>(std::max<unsigned __int128>(1, (span + w - 1) / w));
    };
    s.nb = buckets(s.T0);
    // two backoffs are resolved inside the chunk, so the band region is sized
    // for the backed-off bands as well
    s.n0b[0] = (p.n0 > 0 && p.backoff > 0 && p.n0 - p.backoff > 0) ? p.n0 - p.backoff : 0;
    s.n0b[1] = (s.n0b[0] > 0 && s.n0b[0] - 2 * p.backoff > 0) ? s.n0b[0] - 2 * p.backoff : 0;
    int32_t nb_alloc = s.nb;
    for (int l = 0; l < 2; ++l) {
        s.T0b[l] = s.n0b[l] > 0 ? prefill_key(s.n0b[l], N) : 0;
        s.nbb[l] = s.n0b[l] > 0 ? buckets(s.T0b[l]) : 0;
        nb_alloc = std::max(nb_alloc, s.nbb[l]);
    }
    const double mean = std::ldexp(static_cast<double>(N), shift - 64);
    int cap = static_cast<int>(std::ceil(mean + 8.0 * std::sqrt(mean) + 16.0));
    cap = (cap + 15) / 16 * 16;
    s.cap = std::max(16, std::min(cap, 4096));
    // test hooks: tiny buckets / prefill lists force the redo paths
    if (const char *e = getenv("NZ_DEBUG_BUCKET_CAP")) s.cap = std::max(1, std::min(4096, atoi(e)));
    if (p.n0 > 0) {
        const double e = static_cast<double>(p.n0);
        double want = e + 8.0 * std::sqrt(e) + 64.0;
        if (const char *dbg = getenv("NZ_DEBUG_PREFIX_CAP")) want = std::max(1, atoi(dbg));
        s.prefix_cap = static_cast<int32_t>(std::min<double>(static_cast<double>(N), want * p.prefix_mul));
    } else {
        s.prefix_cap = 0;
    }
    s.par = align_up(static_cast<size_t>(N) * (p.wrap ? 8 : 4));
    s.occ = align_up(static_cast<size_t>((N + 63) / 64) * 8);
    s.keys = align_up(static_cast<size_t>(nb_alloc) * s.cap * 8);
    s.sites = align_up(static_cast<size_t>(nb_alloc) * s.cap * 4);
    s.counts = align_up(static_cast<size_t>(nb_alloc) * 4);
    s.prefix = align_up(static_cast<size_t>(s.prefix_cap) * 4);
    // the bulk labelling's list forest and word positions (not for periodic
    // first-wrap samples, whose labelling runs on the lattice entries)
    s.parc = p.wrap ? 0 : align_up(static_cast<size_t>(s.prefix_cap) * 4);
    s.wpos = (p.wrap || s.prefix_cap == 0) ? 0 : s.occ;
    s.win = p.win_hi > 0 ? align_up(static_cast<size_t>(p.win_hi - p.win_lo) * 4) : 0;
    // bitset summary for the HBM-resident sweep: at most kSumWords words, one
    // bit per 1..16 bitset words (none above that: L > 27, or first-wrap samples)
    {
        const int64_t words = (N + 63) / 64 * 2;
        int gs = 0;
        while (((words >> gs) + 31) / 32 > kSumWords) ++gs;
        s.sum_shift = gs;
        s.sum_words = (gs <= 4 && !p.wrap) ? static_cast<int32_t>(((words >> gs) + 31) / 32 + 1) : 0;
        s.sum = align_up(static_cast<size_t>(s.sum_words) * 4);
    }
    s.total = s.par + s.occ + s.keys + s.sites + s.counts + s.prefix + s.parc + s.wpos + s.win + s.sum;
    return s;
}

// plan_sizes of consecutive plans that share its inputs (the samples of one
// job do) is computed once.
struct SizesMemo {
    bool have = false;
    Plan key{};
    int bucket_log2 = 0;
    Sizes s{};
    const Sizes &get(const Plan &p, int bl)
    {
        if (!have || bl != bucket_log2 || p.L != key.L || p.n0 != key.n0 || p.backoff != key.backoff ||
            p.band_hi != key.band_hi || p.shift_adj != key.shift_adj || p.prefix_mul != key.prefix_mul ||
            p.wrap != key.wrap || p.win_lo != key.win_lo || p.win_hi != key.win_hi) {
            s = plan_sizes(p, bl);
            key = p;
            bucket_log2 = bl;
            have = true;
        }
        return s;
    }
};

int64_t default_band_hi(int32_t L, uint32_t mask, int64_t n0)
{
    const int64_t N = pow5(L);
    if (N <= 8192) return N;
    const int z = coordination(mask);
    const double frac = pc_prior(z) * (1.0 + 4.0 / std::sqrt(static_cast<double>(L)));
    int64_t hi = static_cast<int64_t>(frac * N) + 4096;
    hi = std::max(hi, n0 + 4096);
    return std::min(hi, N);
}

size_t header_bytes(size_t table_entries, int32_t chunk)
{
    return align_up(table_entries * sizeof(NzOffset)) + align_up(chunk * sizeof(NzSample)) +
           align_up(chunk * sizeof(NzState)) + 3 * align_up(chunk * sizeof(int32_t)) + kAlign;
}

struct Tune {
    int residency = 0;
    int wg_waves = 0;
    int waves_per_simd = 0;
    int bucket_log2 = 7;   // mean keys per sort bucket: 128 (256 measured slower at L = 16, 64 no faster)
    int dcap = 64;
    int sweep_mode = 0;
    int summary = 0;
    int split_z = 0;     // widest neighbourhood of the first of two groups side by side (0: kSplitZ)
    // keys launch: one workgroup per block of sites (false), or half as many
    // workgroups as the CUs hold at once, each looping over blocks (true)
    bool keys_resident = false;
};

int check_job(const nz_job &j, int idx)
{
    if (j.L < 1 || j.L > 55) return fail(j.L < 1 ? NZ_EINVAL : NZ_EUNSUPPORTED, "job %d: L = %d outside [1, 55]", idx, j.L);
    if (j.zone_mask < 1 || j.zone_mask > 127) return fail(NZ_EINVAL, "job %d: zone_mask %u outside [1, 127]", idx, j.zone_mask);
    if (j.boundary != NZ_FREE && j.boundary != NZ_PERIODIC)
        return fail(NZ_EINVAL, "job %d: boundary %d is neither NZ_FREE nor NZ_PERIODIC", idx, j.boundary);
    if (j.boundary == NZ_PERIODIC && j.L < 5)
        return fail(NZ_EUNSUPPORTED, "job %d: periodic boundaries need L >= 5", idx);
    if (j.nsamples < 0) return fail(NZ_EINVAL, "job %d: nsamples < 0", idx);
    if (j.sample0 < 0) return fail(NZ_EINVAL, "job %d: sample0 < 0", idx);
    const int64_t N = pow5(j.L);
    if (j.n0 < -1 || j.n0 >= N) return fail(NZ_EINVAL, "job %d: n0 = %lld outside [-1, N-1]", idx, (long long)j.n0);
    if (j.backoff < 0) return fail(NZ_EINVAL, "job %d: backoff < 0", idx);
    if (j.band_hi < 0) return fail(NZ_EINVAL, "job %d: band_hi < 0", idx);
    return NZ_OK;
}

int read_tune(const nz_tuning *t, Tune &out)
{
    out = Tune{};
    if (!t) return NZ_OK;
    if (t->residency < 0 || t->residency > 3) return fail(NZ_EINVAL, "tuning: residency %d outside [0, 3]", t->residency);
    if (t->wg_waves < 0 || t->wg_waves > 4) return fail(NZ_EINVAL, "tuning: wg_waves %d outside [0, 4]", t->wg_waves);
    if (t->waves_per_simd < 0 || t->waves_per_simd > 8)
        return fail(NZ_EINVAL, "tuning: waves_per_simd %d outside [0, 8]", t->waves_per_simd);
    if (t->bucket_log2 != 0 && (t->bucket_log2 < 4 || t->bucket_log2 > 10))
        return fail(NZ_EINVAL, "tuning: bucket_log2 %d outside [4, 10]", t->bucket_log2);
    if (t->sweep_mode < 0 || t->sweep_mode > 2) return fail(NZ_EINVAL, "tuning: sweep_mode %d outside [0, 2]", t->sweep_mode);
    out.sweep_mode = t->sweep_mode;
    if (t->summary < 0 || t->summary > 2) return fail(NZ_EINVAL, "tuning: summary %d outside [0, 2]", t->summary);
    out.summary = t->summary;
    if (t->split_z != 0 && (t->split_z < 10 || t->split_z > 892))
        return fail(NZ_EINVAL, "tuning: split_z %d outside [10, 892]", t->split_z);
    out.split_z = t->split_z;
    out.residency = t->residency;
    out.wg_waves = t->wg_waves;
    out.waves_per_simd = t->waves_per_simd;
    if (t->bucket_log2) out.bucket_log2 = t->bucket_log2;
    return NZ_OK;
}

int nch_for(int z)
{
    if (z <= 64) return 1;
    if (z <= 128) return 2;
    if (z <= 256) return 4;
    if (z <= 512) return 8;
    return 14;
}

// Debug override of the earlier roots one block may touch (tests force the
// block sweep's one-site-at-a-time fallback).
int env_blk_old()
{
    const char *e = getenv("NZ_DEBUG_BLOCK_OLD");
    if (!e) return 256;
    int v = atoi(e);
    return std::max(0, std::min(256, v));
}

// Debug override of the distinct-root list size (tests force early merges).
int env_dcap()
{
    const char *e = getenv("NZ_DEBUG_DCAP");
    if (!e) return 64;
    int v = atoi(e);
    return std::max(2, std::min(64, v));
}

// ---------------------------------------------------------------------------
// The batch engine.

struct TablePool {
    std::map<std::pair<uint32_t, int32_t>, int32_t> index;
    std::vector<NzOffset> entries;
    int32_t get(uint32_t mask, int32_t L, int32_t *z)
    {
        auto key = std::make_pair(mask, L);
        auto it = index.find(key);
        if (it != index.end()) {
            *z = coordination(mask);
            return it->second;
        }
        auto t = build_table(mask, L);
        const int32_t at = static_cast<int32_t>(entries.size());
        entries.insert(entries.end(), t.begin(), t.end());
        index[key] = at;
        *z = static_cast<int32_t>(t.size());
        return at;
    }
};

// smax mode of a whole batch: every sample records S_max(n) for n in
// [win_lo, win_hi) and the chunks add the windows of their samples into out.
struct SmaxReq {
    int64_t win_lo, win_hi;
    uint64_t *d_out;
};

// job_out (may be NULL): first output index of every job (default: the
// samples of the jobs in order, from 0).
int run_batch(const nz_job *jobs, int32_t njobs, uint8_t *ws, size_t ws_bytes, int32_t *d_nstar, int32_t *d_mass,
              int32_t *h_backoffs, const Tune &tune, hipStream_t st, const SmaxReq *smax = nullptr,
              const int64_t *job_out = nullptr)
{
    Device dev;
    if (int rc = device_info(dev)) return rc;
    for (int k = 0; k < 6; ++k) g_stats[k] = 0;
    for (int k = 0; k < 6; ++k) g_ms[k] = 0.0;
    for (int k = 0; k < 5; ++k) g_cc_ms[k] = 0.0;
    g_job_serial.assign(static_cast<size_t>(std::max(njobs, 0)), 0);
    g_job_pre.assign(static_cast<size_t>(std::max(njobs, 0)), 0);
    if (h_backoffs)
        for (int j = 0; j < njobs; ++j) h_backoffs[j] = 0;

    // tables for every (mask, L) of the batch live at the start of the workspace
    TablePool pool;
    std::vector<Plan> todo;
    {
        int64_t total = 0;
        for (int j = 0; j < njobs; ++j) total += std::max<int64_t>(0, jobs[j].nsamples);
        todo.reserve(static_cast<size_t>(std::min<int64_t>(total, 0x7FFFFFFF)));
    }
    int64_t out = 0;
    for (int j = 0; j < njobs; ++j) {
        const nz_job &J = jobs[j];
        int32_t z = 0;
        pool.get(J.zone_mask, J.L, &z);
        const int64_t N = pow5(J.L);
        for (int64_t k = 0; k < J.nsamples; ++k) {
            Plan p{};
            p.job = j;
            p.sample = J.sample0 + k;
            p.out = static_cast<int32_t>(job_out ? job_out[j] + k : out);
            ++out;
            p.L = J.L;
            p.mask = J.zone_mask;
            p.n0 = J.n0 > 0 ? J.n0 : 0;
            p.backoff = J.backoff;
            p.band_hi = J.band_hi > 0 ? std::min<int64_t>(J.band_hi, N) : default_band_hi(J.L, J.zone_mask, p.n0);
            if (p.band_hi <= p.n0) p.band_hi = std::min<int64_t>(N, p.n0 + 4096);
            p.shift_adj = 0;
            p.prefix_mul = 1;
            p.prio = J.prio > 0 ? J.prio : static_cast<double>(std::max<int64_t>(1, p.band_hi - p.n0)) * (1.0 + z / 64.0);
            p.win_lo = smax ? smax->win_lo : 0;
            p.win_hi = smax ? smax->win_hi : 0;
            p.per = J.boundary == NZ_PERIODIC;
            p.wrap = p.per && !smax;
            todo.push_back(p);
        }
    }
    if (out > 0x7FFFFFFF || (job_out && njobs > 0 && job_out[njobs - 1] + jobs[njobs - 1].nsamples > 0x7FFFFFFF))
        return fail(NZ_EINVAL, "too many samples in one batch");
    const size_t tab_bytes = align_up(pool.entries.size() * sizeof(NzOffset));

    int rounds = 0;
    while (!todo.empty()) {
        if (++rounds > 64) return fail(NZ_EDEVICE, "samples still unfinished after 64 redo rounds");
        // free-boundary samples first, then the periodic ones: a chunk holds one
        // boundary condition only, since the sweep is compiled for each
        std::stable_sort(todo.begin(), todo.end(), [](const Plan &a, const Plan &b) {
            return a.per != b.per ? b.per : a.prio > b.prio;
        });
        std::vector<Plan> redo;
        SizesMemo memo;
        size_t pos = 0;
        while (pos < todo.size()) {
            // ---- form a chunk: longest first, as many as the workspace holds
            const int32_t cmax = static_cast<int32_t>(std::min<size_t>(kMaxChunk, todo.size() - pos));
            const size_t head = header_bytes(pool.entries.size(), cmax);
            if (head >= ws_bytes) return fail(NZ_EWORKSPACE, "workspace of %zu bytes is smaller than the %zu-byte header", ws_bytes, head);
            std::vector<Plan> chunk;
            std::vector<Sizes> sizes;
            size_t used = head;
            while (pos < todo.size() && static_cast<int32_t>(chunk.size()) < cmax) {
                if (!chunk.empty() && todo[pos].per != chunk.front().per) break;
                const Sizes &s = memo.get(todo[pos], tune.bucket_log2);
                if (used + s.total > ws_bytes) break;
                used += s.total;
                chunk.push_back(todo[pos]);
                sizes.push_back(s);
                ++pos;
            }
            if (chunk.empty()) {
                Sizes s = plan_sizes(todo[pos], tune.bucket_log2);
                return fail(NZ_EWORKSPACE, "workspace of %zu bytes cannot hold one sample (needs %zu)", ws_bytes, head + s.total);
            }
            ++g_stats[0];
            const int32_t n = static_cast<int32_t>(chunk.size());
            const bool wrap_chunk = chunk.front().wrap;
            const bool per_chunk = chunk.front().per;

            // ---- descriptors, grouped by L for the keys launches
            std::vector<int32_t> byL(n);
            for (int32_t i = 0; i < n; ++i) byL[i] = i;
            std::stable_sort(byL.begin(), byL.end(), [&](int32_t a, int32_t b) { return chunk[a].L < chunk[b].L; });
            std::vector<NzSample> desc(n);
            std::vector<int32_t> out_index(n), queue(n), prefill_list;
            std::vector<int32_t> chunk_of_desc(n);
            size_t off = head;
            int32_t max_nb = 0, max_cap = 0, max_z = 0, max_sum = 0;
            const bool use_sum = tune.summary == 1 || (tune.summary == 0 && n >= kSumSamplesPerCu * dev.cus);
            const int32_t keys_grid = tune.keys_resident ? (nz::keys_resident_wgs() + 1) / 2 * dev.cus : 0;
            uint32_t max_N = 0;
            int64_t max_site = 0;
            std::vector<int32_t> desc_of_chunk(n);
            uint32_t last_mask = 0;   // offset table of the previous descriptor's (mask, L)
            int32_t last_L = 0, last_tab = 0, last_z = 0;
            for (int32_t di = 0; di < n; ++di) {
                const int32_t ci = byL[di];
                const Plan &p = chunk[ci];
                const Sizes &s = sizes[ci];
                const nz_job &J = jobs[p.job];
                NzSample &d = desc[di];
                std::memset(&d, 0, sizeof d);
                d.seed = J.seed;
                d.sample = static_cast<uint64_t>(p.sample);
                d.T0 = s.T0;
                d.L = p.L;
                d.N = static_cast<int32_t>(pow5(p.L));
                d.nb = s.nb;
                d.cap = s.cap;
                d.shift = s.shift;
                d.full = s.full;
                d.prefix_cap = s.prefix_cap;
                if (p.mask != last_mask || p.L != last_L) {
                    last_tab = pool.get(p.mask, p.L, &last_z);
                    last_mask = p.mask;
                    last_L = p.L;
                }
                d.tab = last_tab;
                d.z = last_z;
                d.magic = p.L == 1 ? 0 : static_cast<uint64_t>(~0ull / static_cast<uint64_t>(p.L) + 1ull);
                d.off_par = off; off += s.par;
                d.off_occ = off; off += s.occ;
                d.off_keys = off; off += s.keys;
                d.off_sites = off; off += s.sites;
                d.off_counts = off; off += s.counts;
                d.off_prefix = off; off += s.prefix;
                d.off_parc = off; off += s.parc;
                d.off_wpos = off; off += s.wpos;
                d.off_sum = off; off += s.sum;
                d.sum_shift = s.sum_shift;
                d.sum_words = s.sum_words;
                d.off_win = off; off += s.win;
                d.smax_mode = p.win_hi > 0 ? 1 : 0;
                d.win_lo = static_cast<int32_t>(p.win_lo);
                d.win_hi = static_cast<int32_t>(p.win_hi);
                d.periodic = J.boundary == NZ_PERIODIC ? 1 : 0;
                d.wrap = p.wrap ? 1 : 0;
                out_index[di] = p.out;
                chunk_of_desc[di] = ci;
                desc_of_chunk[ci] = di;
                max_nb = std::max(max_nb, d.nb);
                max_cap = std::max(max_cap, d.cap);
                max_z = std::max(max_z, d.z);
                if (use_sum) max_sum = std::max(max_sum, d.sum_words);
                max_N = std::max(max_N, static_cast<uint32_t>(d.N));
                if (d.T0 != 0) {
                    prefill_list.push_back(di);
                    max_site = std::max<int64_t>(max_site, s.prefix_cap);
                }
            }
            for (int32_t q = 0; q < n; ++q) queue[q] = desc_of_chunk[q];   // chunk is in priority order

            // ---- header layout
            uint8_t *h = ws;
            NzOffset *d_tabs = reinterpret_cast<NzOffset *>(h);
            h += tab_bytes;
            NzSample *d_desc = reinterpret_cast<NzSample *>(h);
            h += align_up(cmax * sizeof(NzSample));
            NzState *d_state = reinterpret_cast<NzState *>(h);
            h += align_up(cmax * sizeof(NzState));
            int32_t *d_queue = reinterpret_cast<int32_t *>(h);
            h += align_up(cmax * sizeof(int32_t));
            int32_t *d_outidx = reinterpret_cast<int32_t *>(h);
            h += align_up(cmax * sizeof(int32_t));
            int32_t *d_list = reinterpret_cast<int32_t *>(h);
            h += align_up(cmax * sizeof(int32_t));
            int32_t *d_qhead = reinterpret_cast<int32_t *>(h);

            HIP_TRY(hipMemcpyAsync(d_tabs, pool.entries.data(), pool.entries.size() * sizeof(NzOffset), hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(d_desc, desc.data(), n * sizeof(NzSample), hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(d_queue, queue.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(d_outidx, out_index.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, st));
            if (!prefill_list.empty())
                HIP_TRY(hipMemcpyAsync(d_list, prefill_list.data(), prefill_list.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
            const int32_t zero = 0;
            HIP_TRY(hipMemcpyAsync(d_qhead, &zero, sizeof zero, hipMemcpyHostToDevice, st));

            // ---- launches
            PhaseEvents *pe = nullptr;
            PrefillEvents *pfe = nullptr;
            if (g_timing) {
                static thread_local PhaseEvents events;   // released when the thread ends
                static thread_local PrefillEvents pevents;
                if (events.ok) pe = &events;
                if (pevents.ok) {
                    pfe = &pevents;
                    pfe->used = 0;
                }
            }
            auto prefill_events = [&]() -> hipEvent_t * {
                return pfe && pfe->used < 3 ? pfe->ev[pfe->used++] : nullptr;
            };
            if (pe) HIP_TRY(hipEventRecord(pe->ev[0], st));
            HIP_TRY(nz::launch_clear(d_desc, nullptr, n, ws, d_state, st));
            for (int32_t a = 0; a < n;) {
                int32_t b = a;
                while (b < n && desc[b].N == desc[a].N) ++b;
                HIP_TRY(nz::launch_keys(d_desc, nullptr, a, b - a, desc[a].N, ws, d_state, keys_grid, st));
                a = b;
            }
            if (pe) HIP_TRY(hipEventRecord(pe->ev[1], st));
            if (!prefill_list.empty()) {
                const int32_t bx_hook = static_cast<int32_t>(std::max<int64_t>(1, std::min<int64_t>(256, (max_site + 1023) / 1024)));
                const int32_t bx_site = static_cast<int32_t>(std::max<int64_t>(1, std::min<int64_t>(1024, (max_site + 1023) / 1024)));
                HIP_TRY(nz::launch_prefill(d_desc, d_list, static_cast<int32_t>(prefill_list.size()), bx_hook, bx_site, d_tabs, ws,
                                           d_state, smax != nullptr, wrap_chunk, per_chunk, st, prefill_events()));
                // Resolve backoffs inside the chunk: samples whose bulk state already
                // spans are re-keyed and re-labelled from n0 - b, and if that spans
                // too from n0 - 3b, so they join this chunk's sweep instead of a
                // later redo round.
                for (int level = 0; level < 2; ++level) {
                    std::vector<NzState> st0(n);
                    HIP_TRY(hipMemcpyAsync(st0.data(), d_state, n * sizeof(NzState), hipMemcpyDeviceToHost, st));
                    HIP_TRY(hipStreamSynchronize(st));
                    std::vector<int32_t> again;
                    for (int32_t di : prefill_list) {
                        if (st0[di].status != NZ_ST_BACKOFF) continue;
                        const int32_t ci = chunk_of_desc[di];
                        const Sizes &s = sizes[ci];
                        if (s.n0b[level] <= 0) continue;   // not planned: the redo round takes it
                        Plan &p = chunk[ci];
                        ++g_stats[3];
                        if (h_backoffs) ++h_backoffs[p.job];
                        p.n0 = s.n0b[level];
                        p.backoff *= 2;   // the next backoff doubles the step
                        desc[di].T0 = s.T0b[level];
                        desc[di].nb = s.nbb[level];
                        max_nb = std::max(max_nb, s.nbb[level]);
                        again.push_back(di);
                    }
                    if (again.empty()) break;
                    std::stable_sort(again.begin(), again.end(), [&](int32_t a, int32_t b) { return desc[a].N < desc[b].N; });
                    const int32_t na = static_cast<int32_t>(again.size());
                    HIP_TRY(hipMemcpyAsync(d_desc, desc.data(), n * sizeof(NzSample), hipMemcpyHostToDevice, st));
                    HIP_TRY(hipMemcpyAsync(d_list, again.data(), na * sizeof(int32_t), hipMemcpyHostToDevice, st));
                    HIP_TRY(nz::launch_clear(d_desc, d_list, na, ws, d_state, st));
                    for (int32_t a = 0; a < na;) {
                        int32_t b = a;
                        while (b < na && desc[again[b]].N == desc[again[a]].N) ++b;
                        HIP_TRY(nz::launch_keys(d_desc, d_list, a, b - a, desc[again[a]].N, ws, d_state, keys_grid, st));
                        a = b;
                    }
                    HIP_TRY(nz::launch_prefill(d_desc, d_list, na, bx_hook, bx_site, d_tabs, ws, d_state, smax != nullptr,
                                               wrap_chunk, per_chunk, st, prefill_events()));
                }
            }
            if (pe) HIP_TRY(hipEventRecord(pe->ev[2], st));
            HIP_TRY(nz::launch_sort(d_desc, n, max_nb, max_cap, ws, st));
            if (pe) HIP_TRY(hipEventRecord(pe->ev[3], st));

            if (wrap_chunk) {
                // periodic first-wrap: one site per step, state in HBM, 4 waves
                // per workgroup
                NzSweepArgs args{};
                args.desc = d_desc;
                args.queue = d_queue;
                args.nqueue = n;
                args.qhead = d_qhead;
                args.tabs = d_tabs;
                args.ws = ws;
                args.state = d_state;
                args.dcap = tune.dcap;
                const int grid = std::max(1, std::min(dev.cus * 8, (n + 3) / 4));
                HIP_TRY(nz::launch_wrap_sweep(nch_for(max_z), args, d_nstar, d_mass, d_outidx, grid, st));
            } else {
                int residency = tune.residency == 3 ? 2 : (tune.residency == 1 ? 1 : 0);
                const uint32_t occ_words = ((max_N + 63) / 64) * 2;
                // HBM residency: the slice starts with the samples' bitset summaries
                uint32_t lds_words = residency == 2 ? occ_words + max_N : (residency == 1 ? occ_words : static_cast<uint32_t>(max_sum));
                // sweep mode: 2 = 64 sites per step for every sample; auto = 64 sites per
                // step for z <= 512 (wider neighbourhoods are faster one site at a time)
                int32_t min_z = 1 << 30;
                for (const NzSample &d : desc) min_z = std::min(min_z, d.z);
                const int32_t blk_zmax = tune.sweep_mode == 2 ? 892 : 512;
                // periodic (largest-cluster) samples go one site per step
                const bool block = !per_chunk && (tune.sweep_mode == 2 || (tune.sweep_mode == 0 && min_z <= blk_zmax));
                if (block) lds_words += nz::block_lds_words();
                int wg_waves = tune.wg_waves ? tune.wg_waves : (residency ? 1 : 4);
                int wps = tune.waves_per_simd ? tune.waves_per_simd : 8;
                size_t lds_wg = static_cast<size_t>(lds_words) * 4 * wg_waves;
                if (lds_wg > dev.lds_per_block)
                    return fail(NZ_EUNSUPPORTED, "residency %d needs %zu bytes of LDS per workgroup; the device allows %zu",
                                tune.residency, lds_wg, dev.lds_per_block);
                int wgs_per_cu = std::max(1, 4 * wps / wg_waves);
                if (lds_wg > 0) wgs_per_cu = std::max<int>(1, std::min<size_t>(wgs_per_cu, dev.lds_per_cu / lds_wg));
                int grid = dev.cus * wgs_per_cu;
                grid = std::min(grid, (n + wg_waves - 1) / wg_waves);
                NzSweepArgs args;
                args.desc = d_desc;
                args.queue = d_queue;
                args.nqueue = n;
                args.qhead = d_qhead;
                args.tabs = d_tabs;
                args.ws = ws;
                args.state = d_state;
                args.lds_words = lds_words;
                args.dcap = tune.dcap;
                args.blk_old = env_blk_old();
                args.blk_zmax = blk_zmax;
                args.use_sum = use_sum ? 1 : 0;
                // the block path's fallback needs more than 8 offset chunks only
                // when a sample wider than z = 512 goes 64 sites per step
                bool wide_block = false;
                for (const NzSample &d : desc) wide_block = wide_block || (block && d.z > 512 && d.z <= blk_zmax && !d.smax_mode);
                HIP_TRY(nz::launch_sweep(nch_for(max_z), wide_block, residency, block, per_chunk, args, d_nstar, d_mass,
                                         d_outidx, grid, wg_waves, st));
            }
            if (smax)
                HIP_TRY(nz::launch_winsum(d_desc, d_state, n, static_cast<int32_t>(smax->win_hi - smax->win_lo), ws,
                                          smax->d_out, st));
            if (pe) HIP_TRY(hipEventRecord(pe->ev[4], st));

            // ---- read back and schedule the redo of unfinished samples
            std::vector<NzState> state(n);
            HIP_TRY(hipMemcpyAsync(state.data(), d_state, n * sizeof(NzState), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (pe) {
                for (int k = 0; k < 4; ++k) {
                    float ms = 0.0f;
                    HIP_TRY(hipEventElapsedTime(&ms, pe->ev[k], pe->ev[k + 1]));
                    g_ms[k] += ms;
                }
                g_ms[5] += 1.0;
            }
            if (pfe) {
                for (int u = 0; u < pfe->used; ++u) {
                    for (int k = 0; k < 4; ++k) {
                        float ms = 0.0f;
                        HIP_TRY(hipEventElapsedTime(&ms, pfe->ev[u][k], pfe->ev[u][k + 1]));
                        g_cc_ms[k] += ms;
                    }
                    g_cc_ms[4] += 1.0;
                }
            }
            if (getenv("NZ_DEBUG_TRACE")) {
                int cnt[8] = {0};
                for (int32_t di = 0; di < n; ++di) ++cnt[std::max(0, std::min(7, static_cast<int>(state[di].status)))];
                std::fprintf(stderr, "nz: round %d chunk of %d: done %d band %d bucket %d backoff %d prefix %d other %d\n",
                             rounds, n, cnt[NZ_ST_DONE], cnt[NZ_ST_BAND], cnt[NZ_ST_BUCKET], cnt[NZ_ST_BACKOFF],
                             cnt[NZ_ST_PREFIX], n - cnt[NZ_ST_DONE] - cnt[NZ_ST_BAND] - cnt[NZ_ST_BUCKET] -
                                                    cnt[NZ_ST_BACKOFF] - cnt[NZ_ST_PREFIX]);
            }
            for (int32_t di = 0; di < n; ++di) {
                Plan p = chunk[chunk_of_desc[di]];
                const int64_t N = pow5(p.L);
                switch (state[di].status) {
                case NZ_ST_DONE:
                    g_stats[4] += state[di].n0;
                    g_stats[5] += (state[di].nstar > 0 ? state[di].nstar : N) - state[di].n0;
                    g_job_pre[p.job] += state[di].n0;
                    g_job_serial[p.job] += (state[di].nstar > 0 ? state[di].nstar : N) - state[di].n0;
                    continue;
                case NZ_ST_BAND:
                    ++g_stats[1];
                    p.band_hi = std::min<int64_t>(N, p.n0 + 2 * std::max<int64_t>(p.band_hi - p.n0, 2048));
                    break;
                case NZ_ST_BUCKET:
                    ++g_stats[2];
                    p.shift_adj += 1;
                    break;
                case NZ_ST_BACKOFF:
                    ++g_stats[3];
                    if (h_backoffs) ++h_backoffs[p.job];
                    // back off by the caller's step, doubling it each time
                    // (n0 - b, n0 - 3b, n0 - 7b, ...), until the start would
                    // reach 0; without a step, halve.  A badly predicted lattice
                    // needs only a few rounds, and n0 reaches 0 after at most
                    // log2(N) of them.
                    if (p.backoff > 0) {
                        if (p.n0 - p.backoff > 0) {
                            p.n0 -= p.backoff;
                            p.backoff *= 2;
                        } else {
                            p.n0 = 0;
                            p.backoff = 0;
                        }
                    } else {
                        p.n0 = p.n0 >= 64 ? p.n0 / 2 : 0;
                    }
                    break;
                case NZ_ST_PREFIX:
                    p.prefix_mul *= 2;
                    break;
                default:
                    return fail(NZ_EDEVICE, "sample %lld finished with status %d", (long long)p.sample, state[di].status);
                }
                redo.push_back(p);
            }
        }
        todo.swap(redo);
    }
    return NZ_OK;
}

size_t batch_bytes(const nz_job *jobs, int32_t njobs, const Tune &tune)
{
    // all samples of the first chunk resident, plus room for one redo of the
    // largest sample with a full band
    std::vector<std::pair<size_t, int64_t>> per;   // (bytes of one sample, samples) of every job
    std::vector<std::pair<uint32_t, int32_t>> tables;
    size_t tab_entries = 0;
    int32_t maxL = 1;
    bool any_wrap = false;
    for (int j = 0; j < njobs; ++j) {
        const auto key = std::make_pair(jobs[j].zone_mask, jobs[j].L);
        if (std::find(tables.begin(), tables.end(), key) == tables.end()) {
            tables.push_back(key);
            tab_entries += static_cast<size_t>(coordination(jobs[j].zone_mask));
        }
        any_wrap = any_wrap || jobs[j].boundary == NZ_PERIODIC;
        Plan p{};
        p.L = jobs[j].L;
        p.mask = jobs[j].zone_mask;
        p.n0 = jobs[j].n0 > 0 ? jobs[j].n0 : 0;
        p.backoff = jobs[j].backoff;   // sizes the band of a first backoff too
        p.wrap = jobs[j].boundary == NZ_PERIODIC;
        const int64_t N = pow5(p.L);
        p.band_hi = jobs[j].band_hi > 0 ? std::min<int64_t>(jobs[j].band_hi, N) : default_band_hi(p.L, p.mask, p.n0);
        if (p.band_hi <= p.n0) p.band_hi = std::min<int64_t>(N, p.n0 + 4096);
        p.prefix_mul = 1;
        if (jobs[j].nsamples > 0) per.emplace_back(plan_sizes(p, tune.bucket_log2).total, jobs[j].nsamples);
        maxL = std::max(maxL, jobs[j].L);
    }
    // the kMaxChunk largest samples
    std::sort(per.begin(), per.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
    int64_t count = 0;
    size_t sum = 0;
    for (const auto &e : per) {
        const int64_t take = std::min<int64_t>(e.second, kMaxChunk - count);
        sum += e.first * static_cast<size_t>(take);
        count += take;
        if (count == kMaxChunk) break;
    }
    size_t total = header_bytes(tab_entries, static_cast<int32_t>(std::max<int64_t>(count, 1))) + sum;
    Plan full{};
    full.L = maxL;
    full.mask = 127;
    full.band_hi = pow5(maxL);
    full.prefix_mul = 1;
    full.wrap = any_wrap;
    total += plan_sizes(full, tune.bucket_log2).total;
    return total;
}

}  // namespace

namespace nz {
int set_error(int code, const char *msg) { return fail(code, "%s", msg); }

int check_batch_fits(const nz_job *jobs, int32_t njobs, const nz_tuning *tune, size_t ws_bytes)
{
    if (njobs < 0 || (njobs > 0 && !jobs)) return fail(NZ_EINVAL, "bad job array");
    for (int j = 0; j < njobs; ++j)
        if (int rc = check_job(jobs[j], j)) return rc;
    Tune t;
    if (int rc = read_tune(tune, t)) return rc;
    try {
        // a chunk's header (sized for as many samples as the batch engine puts
        // in one chunk) plus the largest single sample of any job, planned as
        // the engine plans it
        std::vector<std::pair<uint32_t, int32_t>> tables;
        size_t tab_entries = 0, largest = 0;
        int64_t total = 0;
        int32_t worst = -1;
        for (int j = 0; j < njobs; ++j) {
            const nz_job &J = jobs[j];
            if (J.nsamples <= 0) continue;
            total += J.nsamples;
            const auto key = std::make_pair(J.zone_mask, J.L);
            if (std::find(tables.begin(), tables.end(), key) == tables.end()) {
                tables.push_back(key);
                tab_entries += static_cast<size_t>(coordination(J.zone_mask));
            }
            Plan p{};
            p.L = J.L;
            p.mask = J.zone_mask;
            p.n0 = J.n0 > 0 ? J.n0 : 0;
            p.backoff = J.backoff;
            p.per = J.boundary == NZ_PERIODIC;
            p.wrap = p.per;
            const int64_t N = pow5(J.L);
            p.band_hi = J.band_hi > 0 ? std::min<int64_t>(J.band_hi, N) : default_band_hi(J.L, J.zone_mask, p.n0);
            if (p.band_hi <= p.n0) p.band_hi = std::min<int64_t>(N, p.n0 + 4096);
            p.prefix_mul = 1;
            const size_t b = plan_sizes(p, t.bucket_log2).total;
            if (b > largest) {
                largest = b;
                worst = j;
            }
        }
        if (worst < 0) return NZ_OK;
        const size_t need = header_bytes(tab_entries, static_cast<int32_t>(std::min<int64_t>(total, kMaxChunk))) + largest;
        if (need > ws_bytes)
            return fail(NZ_EWORKSPACE, "job %d (L = %d) needs %zu bytes for one sample; the buffer holds %zu",
                        worst, jobs[worst].L, need, ws_bytes);
    } catch (...) {
        return fail(NZ_ENOMEM, "host allocation failed while sizing the batch");
    }
    return NZ_OK;
}

int run_batch_one_group(const nz_job *jobs, int32_t njobs, uint8_t *ws, size_t ws_bytes, int32_t *d_nstar,
                        int32_t *d_mass, int32_t *h_backoffs, const nz_tuning *tune, hipStream_t st)
{
    int64_t total = 0;
    for (int j = 0; j < njobs; ++j) total += jobs[j].nsamples;
    if (total == 0) {
        for (int k = 0; k < 6; ++k) g_stats[k] = 0;
        if (h_backoffs)
            for (int j = 0; j < njobs; ++j) h_backoffs[j] = 0;
        return NZ_OK;
    }
    if (!d_nstar) return fail(NZ_EINVAL, "n* output is NULL");
    Tune t;
    if (int rc = read_tune(tune, t)) return rc;
    t.dcap = env_dcap();
    // no phase events: this path creates no runtime objects
    const bool timing = g_timing;
    g_timing = false;
    int rc;
    try {
        rc = run_batch(jobs, njobs, ws, ws_bytes, d_nstar, d_mass, h_backoffs, t, st);
    } catch (...) {
        rc = fail(NZ_ENOMEM, "host allocation failed");
    }
    g_timing = timing;
    return rc;
}
}  // namespace nz

// ---------------------------------------------------------------------------
// Public entry points.

NZ_API const char *nz_last_error(void) { return g_err.c_str(); }

NZ_API int nz_abi_version(void) { return NZ_ABI_VERSION; }

NZ_API int nz_coordination(uint32_t zone_mask)
{
    if (zone_mask < 1 || zone_mask > 127) return -1;
    return coordination(zone_mask);
}

NZ_API int nz_last_batch_stats(int64_t stats[6])
{
    if (!stats) return fail(NZ_EINVAL, "stats is NULL");
    for (int k = 0; k < 6; ++k) stats[k] = g_stats[k];
    return NZ_OK;
}

NZ_API int nz_last_batch_job_stats(int64_t *serial, int64_t *prefilled, int32_t njobs)
{
    if (njobs < 0 || (njobs > 0 && (!serial || !prefilled))) return fail(NZ_EINVAL, "NULL output or njobs < 0");
    if (static_cast<size_t>(njobs) != g_job_serial.size())
        return fail(NZ_EINVAL, "the last batch had %zu jobs, not %d", g_job_serial.size(), njobs);
    for (int32_t j = 0; j < njobs; ++j) {
        serial[j] = g_job_serial[j];
        prefilled[j] = g_job_pre[j];
    }
    return NZ_OK;
}

NZ_API int nz_last_batch_cc_timing(double ms[5])
{
    if (!ms) return fail(NZ_EINVAL, "ms is NULL");
    for (int k = 0; k < 5; ++k) ms[k] = g_cc_ms[k];
    return NZ_OK;
}

NZ_API int nz_set_timing(int enable)
{
    g_timing = enable != 0;
    return NZ_OK;
}

NZ_API int nz_last_batch_timing(double ms[6])
{
    if (!ms) return fail(NZ_EINVAL, "ms is NULL");
    for (int k = 0; k < 6; ++k) ms[k] = g_ms[k];
    return NZ_OK;
}

// ---------------------------------------------------------------------------
// Two groups at once.  Narrow neighbourhoods (z <= 64) spend their sweep in
// long chains of dependent 64-site steps that keep few waves busy; a batch that
// also holds wider ones runs the two groups side by side (the wide group on a
// second host thread and stream), so that one group's sweep overlaps the
// other's keys and labelling.  Each group gets its own share of the workspace.

// (256 rather than 512: the L = 24 table of 27 masks x 200 has 400 narrow
// samples, and split it runs 163-167 ms instead of 170-174 learned, 333 ms
// instead of 345-404 plain)
constexpr int64_t kSplitMinSamples = 256;
// widest neighbourhood of the first group (L = 16, 7 compact masks x 1000,
// learned: 47.0 ms with z <= 64, 47.5 with z <= 130, 49.9 with z <= 220;
// with the keys launches keeping their slots: 43.0 ms with z <= 64, 44.1 with
// z <= 10, 45.7 with z <= 130)
constexpr int32_t kSplitZ = 64;

struct SplitPlan {
    std::vector<nz_job> job[2];
    std::vector<int32_t> index[2];   // caller's job index of every job of a group
    std::vector<int64_t> out[2];     // first output index of every job of a group
    size_t bytes[2] = {0, 0};
};

bool split_groups(const nz_job *jobs, int32_t njobs, const Tune &tune, SplitPlan &sp)
{
    if (getenv("NZ_DEBUG_NO_SPLIT")) return false;
    int64_t o = 0, count[2] = {0, 0};
    for (int j = 0; j < njobs; ++j) {
        const int g = coordination(jobs[j].zone_mask) <= (tune.split_z ? tune.split_z : kSplitZ) ? 0 : 1;
        if (jobs[j].nsamples > 0) {
            sp.job[g].push_back(jobs[j]);
            sp.index[g].push_back(j);
            sp.out[g].push_back(o);
            count[g] += jobs[j].nsamples;
        }
        o += jobs[j].nsamples;
    }
    if (count[0] < kSplitMinSamples || count[1] < kSplitMinSamples) return false;
    for (int g = 0; g < 2; ++g) sp.bytes[g] = batch_bytes(sp.job[g].data(), static_cast<int32_t>(sp.job[g].size()), tune);
    return true;
}

// The second group's stream, its start event and host thread live per host
// thread and device.
struct SideStream {
    hipStream_t st = nullptr;
    hipEvent_t start = nullptr;
    bool ok = false;
};

SideStream *side_stream(int device)
{
    static thread_local std::map<int, SideStream> per_device;
    SideStream &s = per_device[device];
    if (!s.ok && !s.st)
        s.ok = hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking) == hipSuccess &&
               hipEventCreateWithFlags(&s.start, hipEventDisableTiming) == hipSuccess;
    return s.ok ? &s : nullptr;
}

int run_split(SplitPlan &sp, int32_t njobs, uint8_t *ws, size_t ws_bytes, int32_t *d_nstar, int32_t *d_mass,
              int32_t *h_backoffs, const Tune &tune, hipStream_t st)
{
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    SideStream *side = side_stream(device);
    if (!side) return fail(NZ_EDEVICE, "could not create the second stream");
    // workspace shares in proportion to the groups' resident sizes
    const size_t wa = static_cast<size_t>(static_cast<long double>(ws_bytes) * sp.bytes[0] /
                                          (sp.bytes[0] + sp.bytes[1])) / kAlign * kAlign;
    std::vector<int32_t> back[2];
    for (int g = 0; g < 2; ++g) back[g].assign(sp.job[g].size(), 0);
    // Side by side, each group's keys launch keeps the CU slots it is given:
    // with a workgroup per block of sites, the short keys workgroups would hand
    // their slots one by one to the other group's long-lived labelling and
    // sweep workgroups (L = 16 learned step: 46.5 -> 43.0 ms with all the
    // slots a CU holds, 42.7 ms with half of them, which leaves the other
    // group's labelling room; a batch that runs as one group is faster with a
    // workgroup per block).
    Tune ts = tune;
    ts.keys_resident = true;
    // the second group starts after the work already queued on the caller's stream
    HIP_TRY(hipEventRecord(side->start, st));
    HIP_TRY(hipStreamWaitEvent(side->st, side->start, 0));
    int rc_b = NZ_OK;
    std::string err_b;
    int64_t stats_b[6] = {0, 0, 0, 0, 0, 0};
    double ms_b[6] = {0, 0, 0, 0, 0, 0};
    double cc_b[5] = {0, 0, 0, 0, 0};
    std::vector<int64_t> serial_b, pre_b;
    const bool timing = g_timing;
    std::thread worker([&]() {
        try {
            if (hipSetDevice(device) != hipSuccess) {
                rc_b = fail(NZ_EDEVICE, "hipSetDevice failed on the second thread");
            } else {
                g_timing = timing;
                rc_b = run_batch(sp.job[1].data(), static_cast<int32_t>(sp.job[1].size()), ws + wa, ws_bytes - wa,
                                 d_nstar, d_mass, back[1].data(), ts, side->st, nullptr, sp.out[1].data());
            }
        } catch (...) {
            rc_b = fail(NZ_ENOMEM, "host allocation failed");
        }
        if (rc_b != NZ_OK) err_b = g_err;
        for (int k = 0; k < 6; ++k) {
            stats_b[k] = g_stats[k];
            ms_b[k] = g_ms[k];
        }
        for (int k = 0; k < 5; ++k) cc_b[k] = g_cc_ms[k];
        serial_b = g_job_serial;
        pre_b = g_job_pre;
    });
    int rc_a;
    try {
        rc_a = run_batch(sp.job[0].data(), static_cast<int32_t>(sp.job[0].size()), ws, wa, d_nstar, d_mass,
                         back[0].data(), ts, st, nullptr, sp.out[0].data());
    } catch (...) {
        rc_a = fail(NZ_ENOMEM, "host allocation failed");
    }
    worker.join();
    for (int k = 0; k < 6; ++k) {
        g_stats[k] += stats_b[k];
        g_ms[k] += ms_b[k];
    }
    for (int k = 0; k < 5; ++k) g_cc_ms[k] += cc_b[k];
    {
        // per-job figures back in the caller's job order
        std::vector<int64_t> serial(static_cast<size_t>(njobs), 0), pre(static_cast<size_t>(njobs), 0);
        for (size_t k = 0; k < sp.job[0].size() && k < g_job_serial.size(); ++k) {
            serial[sp.index[0][k]] = g_job_serial[k];
            pre[sp.index[0][k]] = g_job_pre[k];
        }
        for (size_t k = 0; k < sp.job[1].size() && k < serial_b.size(); ++k) {
            serial[sp.index[1][k]] = serial_b[k];
            pre[sp.index[1][k]] = pre_b[k];
        }
        g_job_serial.swap(serial);
        g_job_pre.swap(pre);
    }
    if (rc_a != NZ_OK) return rc_a;
    if (rc_b != NZ_OK) return fail(rc_b, "%s", err_b.c_str());
    if (h_backoffs) {
        for (int j = 0; j < njobs; ++j) h_backoffs[j] = 0;
        for (int g = 0; g < 2; ++g)
            for (size_t k = 0; k < sp.job[g].size(); ++k) h_backoffs[sp.index[g][k]] = back[g][k];
    }
    return NZ_OK;
}

NZ_API int nz_batch_workspace_bytes(const nz_job *jobs, int32_t njobs, const nz_tuning *tune, size_t *bytes)
{
    if (!bytes) return fail(NZ_EINVAL, "bytes is NULL");
    if (njobs < 0 || (njobs > 0 && !jobs)) return fail(NZ_EINVAL, "bad job array");
    for (int j = 0; j < njobs; ++j)
        if (int rc = check_job(jobs[j], j)) return rc;
    Tune t;
    if (int rc = read_tune(tune, t)) return rc;
    try {
        SplitPlan sp;
        *bytes = split_groups(jobs, njobs, t, sp) ? sp.bytes[0] + sp.bytes[1] + kAlign : batch_bytes(jobs, njobs, t);
    } catch (...) {
        return fail(NZ_ENOMEM, "host allocation failed while sizing the workspace");
    }
    return NZ_OK;
}

NZ_API int nz_sweep_batch(const nz_job *jobs, int32_t njobs, void *d_ws, size_t ws_bytes, int32_t *d_nstar,
                          int32_t *d_mass, int32_t *h_backoffs, const nz_tuning *tune, void *stream)
{
    if (njobs < 0 || (njobs > 0 && !jobs)) return fail(NZ_EINVAL, "bad job array");
    int64_t total = 0;
    for (int j = 0; j < njobs; ++j) {
        if (int rc = check_job(jobs[j], j)) return rc;
        total += jobs[j].nsamples;
    }
    if (total == 0) return NZ_OK;
    if (!d_ws || !d_nstar) return fail(NZ_EINVAL, "workspace or n* output is NULL");
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return fail(NZ_EINVAL, "workspace must be 256-byte aligned");
    Tune t;
    if (int rc = read_tune(tune, t)) return rc;
    // a workspace that cannot hold one sample is refused before any device call
    if (int rc = nz::check_batch_fits(jobs, njobs, tune, ws_bytes)) return rc;
    t.dcap = env_dcap();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (g_timing) {
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        HIP_TRY(hipEventRecord(e0, static_cast<hipStream_t>(stream)));
    }
    int rc;
    try {
        // two groups side by side when the workspace holds both resident
        SplitPlan sp;
        if (split_groups(jobs, njobs, t, sp) && ws_bytes >= sp.bytes[0] + sp.bytes[1] + kAlign)
            rc = run_split(sp, njobs, static_cast<uint8_t *>(d_ws), ws_bytes, d_nstar, d_mass, h_backoffs, t,
                           static_cast<hipStream_t>(stream));
        else
            rc = run_batch(jobs, njobs, static_cast<uint8_t *>(d_ws), ws_bytes, d_nstar, d_mass, h_backoffs, t,
                           static_cast<hipStream_t>(stream));
    } catch (...) {
        rc = fail(NZ_ENOMEM, "host allocation failed");
    }
    if (e0) {
        float ms = 0.0f;
        if (rc == NZ_OK && hipEventRecord(e1, static_cast<hipStream_t>(stream)) == hipSuccess &&
            hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            g_ms[4] = ms;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    return rc;
}

NZ_API int nz_sweep(int32_t L, uint32_t zone_mask, int32_t boundary, int64_t nsamples, uint64_t seed, int32_t *nstar,
                    int32_t *mass)
{
    nz_job j{};
    j.L = L;
    j.zone_mask = zone_mask;
    j.boundary = boundary;
    j.seed = seed;
    j.sample0 = 0;
    j.nsamples = nsamples;
    j.n0 = -1;
    if (int rc = check_job(j, 0)) return rc;
    if (nsamples == 0) return NZ_OK;
    if (!nstar) return fail(NZ_EINVAL, "nstar is NULL");
    if (nsamples > 0x7FFFFFFF) return fail(NZ_EINVAL, "nsamples too large");
    Tune t;
    t.dcap = env_dcap();
    size_t bytes = 0;
    try {
        bytes = batch_bytes(&j, 1, t);
    } catch (...) {
        return fail(NZ_ENOMEM, "host allocation failed");
    }
    // stay well inside the device memory
    size_t freeb = 0, totalb = 0;
    HIP_TRY(hipMemGetInfo(&freeb, &totalb));
    bytes = std::min(bytes, freeb / 2);
    void *ws = nullptr;
    int32_t *dn = nullptr, *dm = nullptr;
    if (hipMalloc(&ws, bytes) != hipSuccess) return fail(NZ_ENOMEM, "hipMalloc of %zu workspace bytes failed", bytes);
    if (hipMalloc(reinterpret_cast<void **>(&dn), nsamples * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&dm), nsamples * 4) != hipSuccess) {
        (void)hipFree(ws);
        (void)hipFree(dn);
        return fail(NZ_ENOMEM, "hipMalloc of outputs failed");
    }
    int rc;
    try {
        rc = run_batch(&j, 1, static_cast<uint8_t *>(ws), bytes, dn, dm, nullptr, t, nullptr);
    } catch (...) {
        rc = fail(NZ_ENOMEM, "host allocation failed");
    }
    if (rc == NZ_OK) {
        if (hipMemcpy(nstar, dn, nsamples * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            (mass && hipMemcpy(mass, dm, nsamples * 4, hipMemcpyDeviceToHost) != hipSuccess))
            rc = fail(NZ_EDEVICE, "copy of results failed");
    }
    (void)hipFree(ws);
    (void)hipFree(dn);
    (void)hipFree(dm);
    return rc;
}

NZ_API int nz_smax_window(int32_t L, uint32_t zone_mask, int32_t boundary, uint64_t seed, int64_t sample0,
                          int64_t nsamples, int64_t n0, int64_t n_lo, int64_t n_hi, uint64_t *smax_sum)
{
    nz_job j{};
    j.L = L;
    j.zone_mask = zone_mask;
    j.boundary = boundary;
    j.seed = seed;
    j.sample0 = sample0;
    j.nsamples = nsamples;
    j.n0 = n0 > 0 ? n0 : -1;
    j.backoff = 0;   // a prefill that reaches the window halves n0
    if (int rc = check_job(j, 0)) return rc;
    const int64_t N = pow5(L);
    if (n_lo < 1 || n_hi <= n_lo || n_hi > N)
        return fail(NZ_EINVAL, "window [%lld, %lld) outside [1, N = %lld]", (long long)n_lo, (long long)n_hi,
                    (long long)N);
    if (n0 >= n_lo) return fail(NZ_EINVAL, "n0 = %lld must lie below the window start %lld", (long long)n0, (long long)n_lo);
    if (!smax_sum) return fail(NZ_EINVAL, "smax_sum is NULL");
    if (nsamples > 0x7FFFFFFF) return fail(NZ_EINVAL, "nsamples too large");
    const int64_t W = n_hi - n_lo;
    for (int64_t k = 0; k < W; ++k) smax_sum[k] = 0;
    if (nsamples == 0) return NZ_OK;
    // the key band ends a little beyond the window, so a band that runs short is rare
    j.band_hi = std::min<int64_t>(N, n_hi + 4 * static_cast<int64_t>(std::sqrt(static_cast<double>(n_hi))) + 1024);
    Tune t;
    t.dcap = env_dcap();
    size_t bytes = 0;
    try {
        bytes = batch_bytes(&j, 1, t) + static_cast<size_t>(std::min<int64_t>(nsamples, kMaxChunk) + 1) *
                                            align_up(static_cast<size_t>(W) * 4);
    } catch (...) {
        return fail(NZ_ENOMEM, "host allocation failed");
    }
    size_t freeb = 0, totalb = 0;
    HIP_TRY(hipMemGetInfo(&freeb, &totalb));
    bytes = std::min(bytes, freeb / 2);
    void *ws = nullptr;
    int32_t *dn = nullptr;
    uint64_t *dsum = nullptr;
    if (hipMalloc(&ws, bytes) != hipSuccess) return fail(NZ_ENOMEM, "hipMalloc of %zu workspace bytes failed", bytes);
    if (hipMalloc(reinterpret_cast<void **>(&dn), nsamples * 4) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&dsum), W * 8) != hipSuccess) {
        (void)hipFree(ws);
        (void)hipFree(dn);
        return fail(NZ_ENOMEM, "hipMalloc of outputs failed");
    }
    int rc = NZ_OK;
    if (hipMemset(dsum, 0, W * 8) != hipSuccess) rc = fail(NZ_EDEVICE, "clearing the window sums failed");
    SmaxReq req{n_lo, n_hi, dsum};
    if (rc == NZ_OK) {
        try {
            rc = run_batch(&j, 1, static_cast<uint8_t *>(ws), bytes, dn, nullptr, nullptr, t, nullptr, &req);
        } catch (...) {
            rc = fail(NZ_ENOMEM, "host allocation failed");
        }
    }
    if (rc == NZ_OK && hipMemcpy(smax_sum, dsum, W * 8, hipMemcpyDeviceToHost) != hipSuccess)
        rc = fail(NZ_EDEVICE, "copy of the window sums failed");
    (void)hipFree(ws);
    (void)hipFree(dn);
    (void)hipFree(dsum);
    return rc;
}

// Binomial convolution of an observable on a window (eqs. (5)-(6) need
// P_max(p) = <S_max(n)>/N convolved with the binomial of (N, p)): the same
// weights as nz_canonical, summed over n in [n_lo, n_hi) only.
NZ_API int nz_convolve_window(const double *Q, int64_t n_lo, int64_t n_hi, int64_t N, const double *p_grid, int64_t np,
                              double *out, double *cover)
{
    if (N < 1 || n_lo < 0 || n_hi > N + 1 || n_lo >= n_hi || !Q)
        return fail(NZ_EINVAL, "window [%lld, %lld) outside [0, N + 1 = %lld]", (long long)n_lo, (long long)n_hi,
                    (long long)(N + 1));
    if (np < 0 || (np > 0 && (!p_grid || !out))) return fail(NZ_EINVAL, "bad p grid or output");
    for (int64_t k = 0; k < np; ++k)
        if (!(p_grid[k] >= 0.0 && p_grid[k] <= 1.0)) return fail(NZ_EINVAL, "p_grid[%lld] outside [0, 1]", (long long)k);
    for (int64_t k = 0; k < np; ++k) {
        const double p = p_grid[k];
        int64_t mode = p == 0.0 ? 0 : (p == 1.0 ? N : static_cast<int64_t>(std::floor((N + 1) * p)));
        if (mode > N) mode = N;
        auto q = [&](int64_t n) { return n >= n_lo && n < n_hi ? Q[n - n_lo] : 0.0; };
        auto in = [&](int64_t n) { return n >= n_lo && n < n_hi ? 1.0 : 0.0; };
        double sw = 1.0, swq = q(mode), swin = in(mode);
        if (p > 0.0 && p < 1.0) {
            const double up = p / (1.0 - p);
            double w = 1.0;
            for (int64_t n = mode; n < N; ++n) {
                w *= static_cast<double>(N - n) / static_cast<double>(n + 1) * up;
                if (w < 1e-300) break;
                sw += w;
                swq += w * q(n + 1);
                swin += w * in(n + 1);
            }
            w = 1.0;
            for (int64_t n = mode; n > 0; --n) {
                w *= static_cast<double>(n) / static_cast<double>(N - n + 1) / up;
                if (w < 1e-300) break;
                sw += w;
                swq += w * q(n - 1);
                swin += w * in(n - 1);
            }
        }
        out[k] = swq / sw;
        if (cover) cover[k] = swin / sw;
    }
    return NZ_OK;
}

// ---------------------------------------------------------------------------
// Learned-prefill planning: the MLP's input rows, its training targets and the
// turn of its outputs into the jobs' prefill depth, backoff step and key band.

// The size input: L enters through the finite-size-scaling variable
// L^(-1/nu), nu = 0.5720 (the 5D correlation-length exponent quoted in
// Sec. II.A.1): the mean of n*/N approaches p_c roughly linearly in it.
constexpr double kNu5 = 0.5720;

double size_variable(int32_t L) { return std::exp(-std::log(static_cast<double>(L)) / kNu5); }

NZ_API int nz_mlp_size_stats(const int32_t *L, int32_t B, double out[2])
{
    if (B < 1 || !L || !out) return fail(NZ_EINVAL, "nz_mlp_size_stats: NULL pointer or B < 1");
    for (int32_t b = 0; b < B; ++b)
        if (L[b] < 1 || L[b] > 55) return fail(NZ_EINVAL, "nz_mlp_size_stats: L[%d] = %d outside [1, 55]", b, L[b]);
    double sum = 0.0;
    for (int32_t b = 0; b < B; ++b) sum += size_variable(L[b]);
    const double mean = sum / B;
    double ss = 0.0;
    for (int32_t b = 0; b < B; ++b) ss += (size_variable(L[b]) - mean) * (size_variable(L[b]) - mean);
    const double sd = std::sqrt(ss / B);
    out[0] = mean;
    out[1] = sd > 0.0 ? sd : 1.0;
    return NZ_OK;
}

NZ_API int nz_mlp_features(const uint32_t *zone_mask, const int32_t *L, int32_t B, double size_mean, double size_std,
                           float *x)
{
    if (B < 1 || !zone_mask || !L || !x) return fail(NZ_EINVAL, "nz_mlp_features: NULL pointer or B < 1");
    if (!(size_std > 0.0)) return fail(NZ_EINVAL, "nz_mlp_features: size_std must be positive");
    for (int32_t b = 0; b < B; ++b) {
        if (zone_mask[b] < 1 || zone_mask[b] > 127 || L[b] < 1 || L[b] > 55)
            return fail(NZ_EINVAL, "nz_mlp_features: row %d has zone_mask %u, L %d", b, zone_mask[b], L[b]);
        for (int k = 0; k < 7; ++k) x[8 * b + k] = static_cast<float>((zone_mask[b] >> k) & 1u);
        x[8 * b + 7] = static_cast<float>((size_variable(L[b]) - size_mean) / size_std);
    }
    return NZ_OK;
}

NZ_API int nz_prefill_target(const int32_t *nstar, int64_t nsamples, int32_t L, double out[5])
{
    if (nsamples < 0 || (nsamples > 0 && !nstar) || !out || L < 1 || L > 55)
        return fail(NZ_EINVAL, "nz_prefill_target: bad arguments");
    const double N = static_cast<double>(pow5(L));
    long double s1 = 0.0L;
    int64_t count = 0;
    for (int64_t k = 0; k < nsamples; ++k)
        if (nstar[k] > 0) {
            s1 += static_cast<long double>(nstar[k]) / N;
            ++count;
        }
    if (count == 0) return fail(NZ_EINVAL, "nz_prefill_target: no sample spans");
    const long double mean = s1 / count;
    long double ss = 0.0L;
    for (int64_t k = 0; k < nsamples; ++k)
        if (nstar[k] > 0) {
            const long double d = static_cast<long double>(nstar[k]) / N - mean;
            ss += d * d;
        }
    const double sd = std::max(static_cast<double>(std::sqrt(ss / count)), 0.5 / N);
    out[0] = static_cast<double>(count);
    out[1] = static_cast<double>(mean);
    out[2] = sd;
    out[3] = std::log(out[1]);
    out[4] = std::log(sd);
    return NZ_OK;
}

NZ_API int nz_prefill_plan(const float *y, nz_job *jobs, int32_t njobs, double k_sigma, double band_sigma,
                           int32_t plain)
{
    if (njobs < 0 || (njobs > 0 && (!y || !jobs))) return fail(NZ_EINVAL, "nz_prefill_plan: NULL pointer or njobs < 0");
    if (!(k_sigma >= 0.0) || !(band_sigma >= 0.0)) return fail(NZ_EINVAL, "nz_prefill_plan: negative sigma factor");
    for (int32_t j = 0; j < njobs; ++j)
        if (jobs[j].L < 1 || jobs[j].L > 55) return fail(NZ_EINVAL, "nz_prefill_plan: job %d has L = %d", j, jobs[j].L);
    for (int32_t j = 0; j < njobs; ++j) {
        nz_job &J = jobs[j];
        const int64_t N = pow5(J.L);
        const double mean = std::exp(static_cast<double>(y[2 * j]));
        const double sd = std::exp(static_cast<double>(y[2 * j + 1]));
        const double hi = std::ceil((mean + band_sigma * sd) * static_cast<double>(N)) + 1024.0;
        J.band_hi = hi >= static_cast<double>(N) ? N : static_cast<int64_t>(hi);
        if (plain) {
            J.n0 = -1;
            continue;
        }
        const double d0 = std::floor((mean - k_sigma * sd) * static_cast<double>(N));
        J.n0 = d0 <= 0.0 ? 0 : (d0 >= static_cast<double>(N - 1) ? N - 1 : static_cast<int64_t>(d0));
        const double b = std::ceil(k_sigma * sd * static_cast<double>(N));
        J.backoff = b >= static_cast<double>(N) ? N : static_cast<int64_t>(b);
    }
    return NZ_OK;
}

// Binomial convolution (Sec. II.B): weights C(N,n) p^n (1-p)^(N-n) are formed
// from the mode outward with the ratio w(n+1)/w(n) = (N-n)/(n+1) * p/(1-p) and
// normalised by their sum.  Terms below 1e-300 of the mode weight are dropped.
NZ_API int nz_canonical(const uint64_t *hist, int64_t hist_len, const double *p_grid, int64_t np, double *R)
{
    if (!hist || hist_len < 2) return fail(NZ_EINVAL, "hist must have at least 2 entries");
    if (np < 0 || (np > 0 && (!p_grid || !R))) return fail(NZ_EINVAL, "bad p grid or output");
    for (int64_t k = 0; k < np; ++k)
        if (!(p_grid[k] >= 0.0 && p_grid[k] <= 1.0)) return fail(NZ_EINVAL, "p_grid[%lld] outside [0, 1]", (long long)k);
    const int64_t N = hist_len - 1;
    std::vector<double> F(N + 1);
    double total = 0.0;
    for (int64_t n = 0; n <= N; ++n) total += static_cast<double>(hist[n]);
    if (total <= 0.0) return fail(NZ_EINVAL, "empty histogram");
    // prefix sums in integers, divided once, so F is exact to rounding
    uint64_t run = 0;
    F[0] = 0.0;
    for (int64_t n = 1; n <= N; ++n) {
        run += hist[n];
        F[n] = static_cast<double>(run) / total;
    }
    for (int64_t k = 0; k < np; ++k) {
        const double p = p_grid[k];
        if (p == 0.0) {
            R[k] = F[0];
            continue;
        }
        if (p == 1.0) {
            R[k] = F[N];
            continue;
        }
        int64_t mode = static_cast<int64_t>(std::floor((N + 1) * p));
        if (mode > N) mode = N;
        const double up = p / (1.0 - p);
        double sw = 1.0, swf = F[mode];
        double w = 1.0;
        for (int64_t n = mode; n < N; ++n) {
            w *= static_cast<double>(N - n) / static_cast<double>(n + 1) * up;
            if (w < 1e-300) break;
            sw += w;
            swf += w * F[n + 1];
        }
        w = 1.0;
        for (int64_t n = mode; n > 0; --n) {
            w *= static_cast<double>(n) / static_cast<double>(N - n + 1) / up;
            if (w < 1e-300) break;
            sw += w;
            swf += w * F[n - 1];
        }
        R[k] = swf / sw;
    }
    return NZ_OK;
}
