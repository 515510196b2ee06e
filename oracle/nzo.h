/*
 * nzo.h -- plain serial CPU oracle for the Newman-Ziff first-spanning sweep on
 * the five-dimensional simple hypercubic lattice sc(5) with complex
 * neighbourhoods (Malarz & Woloszyn, "Random site percolation with complex
 * neighborhoods in five dimension").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load it; the product library never links, includes or calls it, and it
 * shares no source with the product (it has its own zone enumeration, its own
 * Philox, its own sort and its own union-find).
 *
 * What it computes (plain definition; Sec. I for the model, Sec. II.B for the
 * Newman-Ziff construction, eqs. (7)-(8) and Table I for the zones):
 *   - sites i in [0, L^5), coordinates x_j(i) = floor(i / L^j) mod L, x0 fastest;
 *   - the neighbourhood of zone mask m is D(m) = { d in Z^5 : |d|^2 = k, bit k-1
 *     of m set }; zone k is the coordination shell r^2 = k;
 *   - free boundaries: i ~ t iff t = i + d, d in D(m), every coordinate of t
 *     inside [0, L);
 *   - the occupation order is the argsort of 64-bit Philox4x32-10 keys
 *     K(i) (Salmon, Moraes, Dror & Shaw, SC'11), ties broken by site index;
 *   - n* is the first n at which some cluster of the first n sites contains a
 *     site with x0 = 0 and a site with x0 = L-1; mass is that cluster's size;
 *   - periodic boundaries (L >= 5): every coordinate is taken mod L, and n* is
 *     the first n at which some cluster wraps around axis 0, i.e. holds a loop
 *     whose unwrapped x0 displacement is a non-zero multiple of L (Newman &
 *     Ziff 2001, Sec. III); mass is that cluster's size;
 *   - R_L(p) = sum_n C(N,n) p^n (1-p)^(N-n) F_n, the binomial convolution of
 *     Sec. II.B, with F_n the fraction of samples with 1 <= n* <= n.
 */
#ifndef NZO_H
#define NZO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Number of sites of zone k (r^2 = k) in Z^5, k = 1..7; 0 otherwise. */
int nzo_zone_size(int k);

/* Writes the offsets of D(mask) as 5-vectors (d0..d4) into d (capacity 892*5
 * ints) and returns z = |D(mask)|; -1 if mask is outside [1,127]. */
int nzo_offsets(uint32_t mask, int32_t *d);

/* One Philox4x32-10 block: ctr[4], key[2] -> out[4]. */
void nzo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* 64-bit key of site i for (seed, sample) with domain tag 0:
 * key words (lo32(seed), hi32(seed)), counter (floor(i / 2), lo32(sample),
 * hi32(sample), tag); K = (out1 << 32) | out0 for even i, (out3 << 32) | out2
 * for odd i (one Philox block serves two neighbouring sites). */
uint64_t nzo_key(uint64_t seed, uint64_t sample, uint32_t site, uint32_t tag);

/* order[0..n) = indices 0..n-1 sorted ascending by (keys[i], i).  Returns 0 or -1. */
int nzo_sort_keyed(const uint64_t *keys, int64_t n, uint32_t *order);

/* order[0..N) = sites sorted ascending by (K(i), i).  Returns 0 or -1. */
int nzo_order(int32_t L, uint64_t seed, uint64_t sample, uint32_t *order);

/* Serial Newman-Ziff sweep over an explicit order (a permutation prefix of
 * length n_order <= N).  Writes n* (0 = never spans within the order) and the
 * spanning cluster's mass.  If smax is non-NULL it receives the largest cluster
 * size after each step (smax[k] after k+1 sites) for every step performed;
 * if check is non-zero the routine verifies, after every step, that the root
 * sizes sum to the number of occupied sites and that the number of roots equals
 * occupied sites minus successful unions (returns -2 on a violation).
 * run_to_end != 0 keeps adding sites after the first span (for smax).
 * Returns 0, -1 on bad arguments, -2 on an invariant violation. */
int nzo_sweep_order(int32_t L, uint32_t mask, const uint32_t *order, int64_t n_order,
                    int32_t *nstar, int32_t *mass, int32_t *smax, int check, int run_to_end);

/* The same with a boundary choice: periodic != 0 wraps every coordinate mod L
 * (the neighbourhood of a site then always has z members) and n*, mass refer
 * to the first cluster that wraps around axis 0, found from the x0
 * displacement of every site from its parent.  Periodic needs L >= 5. */
int nzo_sweep_order_bc(int32_t L, uint32_t mask, int periodic, const uint32_t *order, int64_t n_order,
                       int32_t *nstar, int32_t *mass, int32_t *smax, int check, int run_to_end);

/* Convenience: keys, sort and sweep for one sample. */
int nzo_sweep(int32_t L, uint32_t mask, uint64_t seed, uint64_t sample,
              int32_t *nstar, int32_t *mass);

/* Many samples (sample0 .. sample0+count-1) spread over nthreads POSIX threads,
 * one sample per thread at a time.  times (may be NULL) receives the summed
 * seconds spent in keys, sort and sweep over all threads. */
int nzo_sweep_many(int32_t L, uint32_t mask, uint64_t seed, uint64_t sample0,
                   int64_t count, int nthreads, int32_t *nstar, int32_t *mass,
                   double times[3]);

/* The same with a boundary choice (periodic != 0: first wrap around axis 0). */
int nzo_sweep_many_bc(int32_t L, uint32_t mask, int periodic, uint64_t seed, uint64_t sample0,
                      int64_t count, int nthreads, int32_t *nstar, int32_t *mass, double times[3]);

/* Cluster labels of the first n sites of the order (label = smallest site index
 * of the cluster; -1 for empty sites), by union-find.  labels has N entries. */
int nzo_prefix_labels(int32_t L, uint32_t mask, const uint32_t *order, int64_t n,
                      int32_t *labels);

/* R_L(p) by binomial convolution in long double (mode-outward weight
 * recurrence).  hist[0] counts samples that never span, hist[n] those with
 * n* = n, hist_len = N + 1. */
int nzo_canonical(const uint64_t *hist, int64_t hist_len, const double *p, int64_t np,
                  double *R);

/* Binomial convolution of an observable Q known for n in [n_lo, n_hi):
 * out[j] = sum_{n_lo <= n < n_hi} B(n; N, p[j]) Q[n - n_lo] and, if cover is
 * non-NULL, cover[j] = sum of the same weights (1 when the window holds the
 * whole binomial mass).  Long double.  Returns 0 or -1. */
int nzo_convolve_window(const double *Q, int64_t n_lo, int64_t n_hi, int64_t N, const double *p, int64_t np,
                        double *out, double *cover);

#ifdef __cplusplus
}
#endif
#endif
