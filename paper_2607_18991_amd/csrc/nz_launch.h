// nz_launch.h -- kernel launchers of nz_kernels.hip used by the host planner.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/nz.h"
#include "nz_internal.h"

namespace nz {

// Samples 0..nsamp-1, or list[0..nsamp) when list != NULL.
hipError_t launch_clear(const NzSample *desc, const int32_t *list, int32_t nsamp, uint8_t *ws, NzState *state,
                        hipStream_t st);

// Keys for samples [first, first + count) of the descriptor array, all of
// lattice size N.
// (list != NULL: samples list[first .. first + count) instead).
// max_grid > 0: at most that many workgroups, each taking several blocks.
// keys_resident_wgs(): workgroups of the keys kernel one CU holds at once.
int32_t keys_resident_wgs();
hipError_t launch_keys(const NzSample *desc, const int32_t *list, int32_t first, int32_t count, int32_t N, uint8_t *ws,
                       NzState *state, int32_t max_grid, hipStream_t st);
int32_t keys_sites_per_block();

hipError_t launch_sort(const NzSample *desc, int32_t nsamp, int32_t max_nb, int32_t max_cap, uint8_t *ws,
                       hipStream_t st);

// Bulk connected components for the samples listed in list[0..nlist).
// smax: also the largest cluster of each smax-mode sample's prefilled state.
// wrap: the listed samples are periodic first-wrap samples (64-bit entries).
// periodic: the listed samples have periodic coordinates (all or none of them).
// ev (may be NULL): five events recorded before the hook, after it, after
// compress and after the size pass, the fifth with the fourth (the size pass
// writes the lattice entries; there is no separate expand pass).
hipError_t launch_prefill(const NzSample *desc, const int32_t *list, int32_t nlist, int32_t bx_hook, int32_t bx_site,
                          const NzOffset *tabs, uint8_t *ws, NzState *state, bool smax, bool wrap, bool periodic,
                          hipStream_t st, hipEvent_t *ev = nullptr);

// out[0..w) += sum over the chunk's finished samples 0..nsamp-1 of their S_max windows.
hipError_t launch_winsum(const NzSample *desc, const NzState *state, int32_t nsamp, int32_t w, const uint8_t *ws,
                         uint64_t *out, hipStream_t st);

// residency: 0 HBM, 1 bitset in LDS, 2 bitset and parents in LDS.
// nch in {1, 2, 4, 8, 14}.  block: 64 sites per wave step (the wave's LDS
// slice must end with block_lds_words() words for the block's site table).
// wide_block: some block sample has z > 512, so the block path's one-site
// fallback needs all nch chunks (else it is compiled for at most 8).
// periodic: every sample of the chunk has periodic coordinates (largest-cluster
// windows); such a chunk goes one site per step (block must be false).
hipError_t launch_sweep(int nch, bool wide_block, int residency, bool block, bool periodic, const NzSweepArgs &a,
                        int32_t *nstar, int32_t *mass, const int32_t *out_index, int grid, int wg_waves, hipStream_t st);
uint32_t block_lds_words();

// Periodic first-wrap sweep of a chunk whose samples all have wrap set; one
// site per step, state in HBM, 256-thread workgroups.
hipError_t launch_wrap_sweep(int nch, const NzSweepArgs &a, int32_t *nstar, int32_t *mass, const int32_t *out_index,
                             int grid, hipStream_t st);

// Host side of nz_sweep_batch_static (nz_api.cpp): whether a chunk header and
// the largest single sample of the jobs fit a buffer of ws_bytes; and
// the batch engine run as one group on one stream with no events, threads or
// streams of its own.
int set_error(int code, const char *msg);
int check_batch_fits(const nz_job *jobs, int32_t njobs, const nz_tuning *tune, size_t ws_bytes);
int run_batch_one_group(const nz_job *jobs, int32_t njobs, uint8_t *ws, size_t ws_bytes, int32_t *d_nstar,
                        int32_t *d_mass, int32_t *h_backoffs, const nz_tuning *tune, hipStream_t st);

}  // namespace nz
