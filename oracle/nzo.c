/*
 * nzo.c -- plain serial CPU oracle (test infrastructure only; see nzo.h).
 *
 * Every routine here is written for a reader to check against the paper by
 * eye: no blocking, no fusion, no clever encodings.  Integers are exact;
 * the binomial convolution runs in long double.
 */
#define _GNU_SOURCE
#include "nzo.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* ------------------------------------------------------------------------ */
/* Zones (Sec. II.A.2, eqs. (7)-(8); zone sizes in the single-zone rows of
 * Table I).  Zone k is the set of lattice vectors d with |d|^2 = k.  In five
 * dimensions every such d has |d_j| <= 2, so scanning {-2..2}^5 is complete. */

int nzo_zone_size(int k)
{
    if (k < 1 || k > 7) return 0;
    int count = 0;
    for (int a = -2; a <= 2; ++a)
        for (int b = -2; b <= 2; ++b)
            for (int c = -2; c <= 2; ++c)
                for (int e = -2; e <= 2; ++e)
                    for (int f = -2; f <= 2; ++f)
                        if (a * a + b * b + c * c + e * e + f * f == k) ++count;
    return count;
}

int nzo_offsets(uint32_t mask, int32_t *d)
{
    if (mask < 1 || mask > 127) return -1;
    int z = 0;
    for (int k = 1; k <= 7; ++k) {
        if (!(mask & (1u << (k - 1)))) continue;
        for (int a = -2; a <= 2; ++a)
            for (int b = -2; b <= 2; ++b)
                for (int c = -2; c <= 2; ++c)
                    for (int e = -2; e <= 2; ++e)
                        for (int f = -2; f <= 2; ++f)
                            if (a * a + b * b + c * c + e * e + f * f == k) {
                                d[5 * z + 0] = a;
                                d[5 * z + 1] = b;
                                d[5 * z + 2] = c;
                                d[5 * z + 3] = e;
                                d[5 * z + 4] = f;
                                ++z;
                            }
    }
    return z;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11, Sec. 4): ten rounds of
 * a multiply-based bijection on four 32-bit words; the two key words are
 * advanced by the Weyl constants (golden ratio, sqrt(3)-1) between rounds. */

static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

void nzo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Sites 2j and 2j + 1 share the Philox block of counter j: the even site takes
 * words (1, 0), the odd site words (3, 2). */
uint64_t nzo_key(uint64_t seed, uint64_t sample, uint32_t site, uint32_t tag)
{
    uint32_t ctr[4] = { site >> 1, (uint32_t)sample, (uint32_t)(sample >> 32), tag };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t out[4];
    nzo_philox4x32_10(ctr, key, out);
    if (site & 1u) return ((uint64_t)out[3] << 32) | (uint64_t)out[2];
    return ((uint64_t)out[1] << 32) | (uint64_t)out[0];
}

/* ------------------------------------------------------------------------ */
/* Occupation order: the sites sorted ascending by (K(i), i). */

typedef struct { uint64_t k; uint32_t i; } keyed_site;

static int cmp_keyed(const void *a, const void *b)
{
    const keyed_site *x = (const keyed_site *)a, *y = (const keyed_site *)b;
    if (x->k < y->k) return -1;
    if (x->k > y->k) return 1;
    if (x->i < y->i) return -1;
    if (x->i > y->i) return 1;
    return 0;
}

int nzo_sort_keyed(const uint64_t *keys, int64_t n, uint32_t *order)
{
    if (n < 0 || (n > 0 && (!keys || !order))) return -1;
    keyed_site *ks = (keyed_site *)malloc((size_t)(n > 0 ? n : 1) * sizeof(keyed_site));
    if (!ks) return -1;
    for (int64_t i = 0; i < n; ++i) { ks[i].k = keys[i]; ks[i].i = (uint32_t)i; }
    qsort(ks, (size_t)n, sizeof(keyed_site), cmp_keyed);
    for (int64_t i = 0; i < n; ++i) order[i] = ks[i].i;
    free(ks);
    return 0;
}

static int64_t ipow5(int32_t L) { return (int64_t)L * L * L * L * L; }

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

static int order_timed(int32_t L, uint64_t seed, uint64_t sample, uint32_t *order,
                       double *t_keys, double *t_sort)
{
    if (L < 1 || L > 55) return -1;
    int64_t N = ipow5(L);
    keyed_site *ks = (keyed_site *)malloc((size_t)N * sizeof(keyed_site));
    if (!ks) return -1;
    double t0 = now_s();
    for (int64_t i = 0; i < N; ++i) {
        ks[i].k = nzo_key(seed, sample, (uint32_t)i, 0);
        ks[i].i = (uint32_t)i;
    }
    double t1 = now_s();
    qsort(ks, (size_t)N, sizeof(keyed_site), cmp_keyed);
    for (int64_t i = 0; i < N; ++i) order[i] = ks[i].i;
    double t2 = now_s();
    free(ks);
    if (t_keys) *t_keys += t1 - t0;
    if (t_sort) *t_sort += t2 - t1;
    return 0;
}

int nzo_order(int32_t L, uint64_t seed, uint64_t sample, uint32_t *order)
{
    return order_timed(L, seed, sample, order, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Union-find in the style of Newman & Ziff (2001): ptr[i] is EMPTY for an
 * unoccupied site, the parent index for a non-root, and minus the cluster size
 * for a root.  Finds compress the whole path; unions attach the smaller
 * cluster below the larger one (equal sizes: the smaller index stays root).
 * flags[root] holds LO (a member has x0 = 0) and HI (a member has x0 = L-1).
 *
 * Periodic boundaries (Newman & Ziff 2001, Sec. III, wrapping clusters): every
 * site also keeps dx[i], its x0 displacement from its parent in the unwrapped
 * lattice (0 at a root), so the displacement of a site from its root is the
 * sum along its path.  An edge s -> t = s + d inside one cluster closes a loop;
 * the loop winds around axis 0 exactly when D(s) + d0 != D(t), and the cluster
 * is then marked LO | HI, the same state a spanning cluster has under free
 * boundaries. */

#define EMPTY INT32_MIN
#define FLAG_LO 1u
#define FLAG_HI 2u

static int32_t uf_find(int32_t *ptr, int32_t i)
{
    int32_t r = i;
    while (ptr[r] >= 0) r = ptr[r];
    while (ptr[i] >= 0) {
        int32_t next = ptr[i];
        ptr[i] = r;
        i = next;
    }
    return r;
}

/* Root of i and, through *disp, the x0 displacement of i from it; the path is
 * compressed with each node's displacement rewritten to be from the root. */
static int32_t uf_find_disp(int32_t *ptr, int32_t *dx, int32_t i, int32_t *disp)
{
    int32_t r = i, total = 0;
    while (ptr[r] >= 0) {
        total += dx[r];
        r = ptr[r];
    }
    *disp = total;
    int32_t rem = total;
    while (ptr[i] >= 0) {
        int32_t next = ptr[i], step = dx[i];
        ptr[i] = r;
        dx[i] = rem;
        rem -= step;
        i = next;
    }
    return r;
}

/* Returns the surviving root. */
static int32_t uf_union(int32_t *ptr, uint8_t *flags, int32_t a, int32_t b)
{
    int32_t sa = -ptr[a], sb = -ptr[b];
    int32_t big = a, small = b;
    if (sb > sa || (sb == sa && b < a)) { big = b; small = a; }
    ptr[big] += ptr[small];      /* both negative: sizes add */
    ptr[small] = big;
    flags[big] |= flags[small];
    return big;
}

static void decode(int32_t L, int64_t i, int32_t x[5])
{
    for (int j = 0; j < 5; ++j) {
        x[j] = (int32_t)(i % L);
        i /= L;
    }
}

/* Neighbour t of s along offset d: free boundaries give -1 when it falls
 * outside the lattice; periodic boundaries take every coordinate mod L. */
static int64_t neighbour(int32_t L, const int32_t xs[5], const int32_t *d, int periodic)
{
    int64_t t = 0, stride = 1;
    for (int j = 0; j < 5; ++j) {
        int32_t y = xs[j] + d[j];
        if (periodic) y = ((y % L) + L) % L;
        else if (y < 0 || y >= L) return -1;
        t += stride * y;
        stride *= L;
    }
    return t;
}

int nzo_sweep_order(int32_t L, uint32_t mask, const uint32_t *order, int64_t n_order,
                    int32_t *nstar, int32_t *mass, int32_t *smax, int check, int run_to_end)
{
    return nzo_sweep_order_bc(L, mask, 0, order, n_order, nstar, mass, smax, check, run_to_end);
}

int nzo_sweep_order_bc(int32_t L, uint32_t mask, int periodic, const uint32_t *order, int64_t n_order,
                       int32_t *nstar, int32_t *mass, int32_t *smax, int check, int run_to_end)
{
    if (L < 1 || L > 55 || mask < 1 || mask > 127 || !order || !nstar || !mass) return -1;
    int64_t N = ipow5(L);
    if (n_order < 0 || n_order > N) return -1;

    int32_t off[892 * 5];
    int z = nzo_offsets(mask, off);

    /* below L = 5 two offsets of one neighbourhood can reach the same site
     * around the torus, and a displacement is no longer fixed by the pair */
    if (periodic && L < 5) return -1;

    int32_t *ptr = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    uint8_t *flags = (uint8_t *)calloc((size_t)N, 1);
    int32_t *dx = periodic ? (int32_t *)calloc((size_t)N, sizeof(int32_t)) : NULL;
    if (!ptr || !flags || (periodic && !dx)) { free(ptr); free(flags); free(dx); return -1; }
    for (int64_t i = 0; i < N; ++i) ptr[i] = EMPTY;

    *nstar = 0;
    *mass = 0;
    int32_t biggest = 0;
    int64_t unions = 0;
    int rc = 0;
    for (int64_t k = 0; k < n_order; ++k) {
        int32_t s = (int32_t)order[k];
        int32_t xs[5];
        decode(L, s, xs);
        ptr[s] = -1;
        /* periodic boundaries have no borders; a cluster there "spans" when it
         * wraps around axis 0 */
        flags[s] = periodic ? 0 : (uint8_t)((xs[0] == 0 ? FLAG_LO : 0) | (xs[0] == L - 1 ? FLAG_HI : 0));
        if (biggest < 1) biggest = 1;

        for (int q = 0; q < z; ++q) {
            int64_t t = neighbour(L, xs, off + 5 * q, periodic);
            if (t < 0 || ptr[t] == EMPTY) continue;
            if (!periodic) {
                int32_t rs = uf_find(ptr, s);
                int32_t rt = uf_find(ptr, (int32_t)t);
                if (rs != rt) {
                    int32_t r = uf_union(ptr, flags, rs, rt);
                    ++unions;
                    if (-ptr[r] > biggest) biggest = -ptr[r];
                }
                continue;
            }
            /* unwrapped: t = s + d, so its x0 is that of s plus d0 */
            int32_t d0 = off[5 * q], Ds, Dt;
            int32_t rs = uf_find_disp(ptr, dx, s, &Ds);
            int32_t rt = uf_find_disp(ptr, dx, (int32_t)t, &Dt);
            if (rs == rt) {
                if (Ds + d0 != Dt) flags[rs] |= FLAG_LO | FLAG_HI;
                continue;
            }
            int32_t r = uf_union(ptr, flags, rs, rt);
            /* the attached root's displacement from the survivor, from
             * x0(rs) = x0(s) - Ds and x0(rt) = x0(s) + d0 - Dt */
            if (r == rt) dx[rs] = Dt - d0 - Ds;
            else dx[rt] = Ds + d0 - Dt;
            ++unions;
            if (-ptr[r] > biggest) biggest = -ptr[r];
        }

        if (smax) smax[k] = biggest;

        if (check) {
            /* Conservation: root sizes sum to k+1, roots = occupied - unions. */
            int64_t sum = 0, roots = 0;
            for (int64_t m = 0; m <= k; ++m) {
                int32_t u = (int32_t)order[m];
                if (ptr[u] < 0) { sum += -ptr[u]; ++roots; }
            }
            if (sum != k + 1 || roots != k + 1 - unions) { rc = -2; break; }
        }

        int32_t dummy;
        int32_t r = periodic ? uf_find_disp(ptr, dx, s, &dummy) : uf_find(ptr, s);
        if (*nstar == 0 && flags[r] == (FLAG_LO | FLAG_HI)) {
            *nstar = (int32_t)(k + 1);
            *mass = -ptr[r];
            if (!run_to_end) break;
        }
    }
    free(ptr);
    free(flags);
    free(dx);
    return rc;
}

int nzo_sweep(int32_t L, uint32_t mask, uint64_t seed, uint64_t sample,
              int32_t *nstar, int32_t *mass)
{
    if (L < 1 || L > 55) return -1;
    int64_t N = ipow5(L);
    uint32_t *order = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    if (!order) return -1;
    int rc = nzo_order(L, seed, sample, order);
    if (rc == 0) rc = nzo_sweep_order(L, mask, order, N, nstar, mass, NULL, 0, 0);
    free(order);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Independent samples over threads: the paper's "ordinary work division"
 * (Sec. II.B), one whole simulation per thread. */

typedef struct {
    int32_t L;
    uint32_t mask;
    int periodic;
    uint64_t seed, sample0;
    int64_t count;
    int64_t next;            /* shared work counter */
    int32_t *nstar, *mass;
    int rc;
    double t_keys, t_sort, t_sweep;
    pthread_mutex_t lock;
} many_ctx;

static void *many_worker(void *arg)
{
    many_ctx *c = (many_ctx *)arg;
    int64_t N = ipow5(c->L);
    uint32_t *order = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
    double tk = 0, ts = 0, tw = 0;
    int rc = order ? 0 : -1;
    while (rc == 0) {
        int64_t k = __atomic_fetch_add(&c->next, 1, __ATOMIC_RELAXED);
        if (k >= c->count) break;
        rc = order_timed(c->L, c->seed, c->sample0 + (uint64_t)k, order, &tk, &ts);
        if (rc) break;
        double t0 = now_s();
        rc = nzo_sweep_order_bc(c->L, c->mask, c->periodic, order, N, &c->nstar[k], &c->mass[k], NULL, 0, 0);
        tw += now_s() - t0;
    }
    free(order);
    pthread_mutex_lock(&c->lock);
    if (rc) c->rc = rc;
    c->t_keys += tk;
    c->t_sort += ts;
    c->t_sweep += tw;
    pthread_mutex_unlock(&c->lock);
    return NULL;
}

int nzo_sweep_many(int32_t L, uint32_t mask, uint64_t seed, uint64_t sample0,
                   int64_t count, int nthreads, int32_t *nstar, int32_t *mass,
                   double times[3])
{
    return nzo_sweep_many_bc(L, mask, 0, seed, sample0, count, nthreads, nstar, mass, times);
}

int nzo_sweep_many_bc(int32_t L, uint32_t mask, int periodic, uint64_t seed, uint64_t sample0,
                      int64_t count, int nthreads, int32_t *nstar, int32_t *mass, double times[3])
{
    if (L < 1 || L > 55 || mask < 1 || mask > 127 || count < 0 || nthreads < 1) return -1;
    if (periodic && L < 5) return -1;
    if (count > 0 && (!nstar || !mass)) return -1;
    many_ctx c;
    memset(&c, 0, sizeof c);
    c.L = L; c.mask = mask; c.periodic = periodic; c.seed = seed; c.sample0 = sample0; c.count = count;
    c.nstar = nstar; c.mass = mass;
    pthread_mutex_init(&c.lock, NULL);
    pthread_t *th = (pthread_t *)malloc((size_t)nthreads * sizeof(pthread_t));
    if (!th) return -1;
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, many_worker, &c);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&c.lock);
    if (times) { times[0] = c.t_keys; times[1] = c.t_sort; times[2] = c.t_sweep; }
    return c.rc;
}

/* ------------------------------------------------------------------------ */

int nzo_prefix_labels(int32_t L, uint32_t mask, const uint32_t *order, int64_t n,
                      int32_t *labels)
{
    if (L < 1 || L > 55 || mask < 1 || mask > 127 || !order || !labels) return -1;
    int64_t N = ipow5(L);
    if (n < 0 || n > N) return -1;
    int32_t off[892 * 5];
    int z = nzo_offsets(mask, off);
    int32_t *ptr = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    uint8_t *flags = (uint8_t *)calloc((size_t)N, 1);
    if (!ptr || !flags) { free(ptr); free(flags); return -1; }
    for (int64_t i = 0; i < N; ++i) ptr[i] = EMPTY;
    for (int64_t k = 0; k < n; ++k) {
        int32_t s = (int32_t)order[k];
        int32_t xs[5];
        decode(L, s, xs);
        ptr[s] = -1;
        for (int q = 0; q < z; ++q) {
            int64_t t = neighbour(L, xs, off + 5 * q, 0);
            if (t < 0 || ptr[t] == EMPTY) continue;
            int32_t rs = uf_find(ptr, s), rt = uf_find(ptr, (int32_t)t);
            if (rs != rt) uf_union(ptr, flags, rs, rt);
        }
    }
    /* label = smallest member index of the cluster */
    int32_t *minidx = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    if (!minidx) { free(ptr); free(flags); return -1; }
    for (int64_t i = 0; i < N; ++i) minidx[i] = INT32_MAX;
    for (int64_t i = 0; i < N; ++i) {
        if (ptr[i] == EMPTY) continue;
        int32_t r = uf_find(ptr, (int32_t)i);
        if ((int32_t)i < minidx[r]) minidx[r] = (int32_t)i;
    }
    for (int64_t i = 0; i < N; ++i)
        labels[i] = (ptr[i] == EMPTY) ? -1 : minidx[uf_find(ptr, (int32_t)i)];
    free(minidx);
    free(ptr);
    free(flags);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Binomial convolution (Sec. II.B): the weights B(n; N, p) are built from the
 * mode outwards by the ratio B(n+1)/B(n) = (N-n)/(n+1) * p/(1-p), then
 * normalised by their sum, so no factorial or log-gamma is ever formed. */

int nzo_canonical(const uint64_t *hist, int64_t hist_len, const double *p, int64_t np,
                  double *R)
{
    if (!hist || hist_len < 2 || np < 0 || (np > 0 && (!p || !R))) return -1;
    int64_t N = hist_len - 1;
    long double total = 0.0L;
    for (int64_t n = 0; n <= N; ++n) total += (long double)hist[n];
    if (total <= 0.0L) return -1;
    long double *F = (long double *)malloc((size_t)(N + 1) * sizeof(long double));
    long double *w = (long double *)malloc((size_t)(N + 1) * sizeof(long double));
    if (!F || !w) { free(F); free(w); return -1; }
    long double run = 0.0L;
    F[0] = 0.0L;                         /* n* = 0 means "never spans" */
    for (int64_t n = 1; n <= N; ++n) {
        run += (long double)hist[n];
        F[n] = run / total;
    }
    int rc = 0;
    for (int64_t j = 0; j < np; ++j) {
        long double q = p[j];
        if (!(q >= 0.0L && q <= 1.0L)) { rc = -1; break; }
        if (q == 0.0L) { R[j] = (double)F[0]; continue; }
        if (q == 1.0L) { R[j] = (double)F[N]; continue; }
        int64_t m = (int64_t)((long double)(N + 1) * q);
        if (m > N) m = N;
        long double ratio_up = q / (1.0L - q);
        w[m] = 1.0L;
        for (int64_t n = m; n < N; ++n)
            w[n + 1] = w[n] * ((long double)(N - n) / (long double)(n + 1)) * ratio_up;
        for (int64_t n = m; n > 0; --n)
            w[n - 1] = w[n] * ((long double)n / (long double)(N - n + 1)) / ratio_up;
        long double sw = 0.0L, swf = 0.0L;
        for (int64_t n = 0; n <= N; ++n) {
            sw += w[n];
            swf += w[n] * F[n];
        }
        R[j] = (double)(swf / sw);
    }
    free(F);
    free(w);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Binomial convolution of an observable known on a window of n: eq. (5)-(6)
 * need P_max(p) = sum_n C(N,n) p^n (1-p)^(N-n) S_max(n) / N; only n in
 * [n_lo, n_hi) are summed.  out[j] = sum_{window} B(n) Q[n - n_lo] and
 * cover[j] = sum_{window} B(n), with B the binomial pmf of (N, p[j]) (weights
 * built outward from the mode by the ratio recurrence, normalised by their sum
 * over 0..N). */
int nzo_convolve_window(const double *Q, int64_t n_lo, int64_t n_hi, int64_t N, const double *p, int64_t np,
                        double *out, double *cover)
{
    if (N < 1 || n_lo < 0 || n_hi > N + 1 || n_lo >= n_hi || !Q || np < 0 || (np > 0 && (!p || !out))) return -1;
    long double *w = (long double *)malloc((size_t)(N + 1) * sizeof(long double));
    if (!w) return -1;
    int rc = 0;
    for (int64_t j = 0; j < np; ++j) {
        long double q = p[j];
        if (!(q >= 0.0L && q <= 1.0L)) { rc = -1; break; }
        for (int64_t n = 0; n <= N; ++n) w[n] = 0.0L;
        if (q == 0.0L) w[0] = 1.0L;
        else if (q == 1.0L) w[N] = 1.0L;
        else {
            int64_t m = (int64_t)((long double)(N + 1) * q);
            if (m > N) m = N;
            long double ratio_up = q / (1.0L - q);
            w[m] = 1.0L;
            for (int64_t n = m; n < N; ++n)
                w[n + 1] = w[n] * ((long double)(N - n) / (long double)(n + 1)) * ratio_up;
            for (int64_t n = m; n > 0; --n)
                w[n - 1] = w[n] * ((long double)n / (long double)(N - n + 1)) / ratio_up;
        }
        long double sw = 0.0L, swq = 0.0L, swin = 0.0L;
        for (int64_t n = 0; n <= N; ++n) sw += w[n];
        for (int64_t n = n_lo; n < n_hi; ++n) {
            swq += w[n] * (long double)Q[n - n_lo];
            swin += w[n];
        }
        out[j] = (double)(swq / sw);
        if (cover) cover[j] = (double)(swin / sw);
    }
    free(w);
    return rc;
}
