/*
 * ksg_oracle.c -- plain brute-force reference for ensemble transfer entropy.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  It shares no code, header, table or constant with the
 * library; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  Nothing here is tuned for speed.
 *
 * What it computes (Wollstadt et al. 2014, "Efficient transfer entropy
 * analysis of non-stationary neural time series"):
 *
 *   embedding   eq. 6-7 and the sentence after them (the source state at t-u is
 *               built like the target past): for repetition r and sample t',
 *               z = ( y_t'(r) | y_{t'-1}(r), ..., y_{t'-1-(d_y-1)tau}(r)
 *                             | x_{t'-u}(r), ..., x_{t'-u-(d_x-1)tau}(r) ).
 *               Points of all repetitions r < R_c and all t' of the window
 *               [w, w+W) are pooled (eq. 10), repetition-major.
 *   surrogates  the repetitions of one process are permuted blockwise, the same
 *               permutation for every t' of the window (Fig. 3 and the
 *               surrogate paragraph of "Main analysis work flow").
 *   search      KSG type-1 with projected distances (text before eq. 9): the
 *               radius eps_i is the max-norm distance to the k-th nearest
 *               neighbour in the joint space, self excluded; the counts n are
 *               the numbers of points strictly closer than eps_i in the spaces
 *               (P), (T,P) and (P,S) of the four-entropy split, eq. 8.
 *   estimate    eq. 9 / eq. 10: TE = psi(k) + < psi(n_P+1) - psi(n_TP+1) - psi(n_PS+1) >.
 *   p-value     the fraction of surrogate estimates equal to or larger than
 *               the original one ("TE calculation and statistical testing").
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   - per-coordinate differences are IEEE binary32 round-to-nearest-even
 *     differences of the float32 data; the oracle forms them exactly in double
 *     and rounds once to float, which is the same binary32 result because
 *     double carries more than 2*24+2 significand bits;
 *   - self is excluded by index only; other points at distance 0 count;
 *   - range counts are strict (<);
 *   - eps is the k-th order statistic of the distance multiset;
 *   - d_y = 0 (no target past) is accepted here only, as a reduction of the
 *     estimator to the KSG mutual-information estimator 1 used as a pin.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ---------------------------------------------------------------- embedding */

/* Build the pooled points of one analysis window as float32 [N][D], D = 1+d_y+d_x,
 * N = Rc*W, point index q = r*W + (t' - w).  src_perm / tgt_perm (length Rc, may be
 * NULL) give the repetition the source / target values of repetition r are read from.
 * Returns 0, or -1 if an index falls outside the series. */
int ksg_embed(const float *x, const float *y, int R, int T,
              int d_y, int d_x, int tau, int u,
              int w, int W, int Rc,
              const int32_t *src_perm, const int32_t *tgt_perm, float *out)
{
    const int D = 1 + d_y + d_x;
    if (Rc > R || Rc < 1 || W < 1 || d_y < 0 || d_x < 1 || tau < 1 || u < 1)
        return -1;
    for (int r = 0; r < Rc; ++r) {
        const int rs = src_perm ? src_perm[r] : r;
        const int rt = tgt_perm ? tgt_perm[r] : r;
        if (rs < 0 || rs >= R || rt < 0 || rt >= R)
            return -1;
        const float *yr = y + (size_t)rt * T;
        const float *xr = x + (size_t)rs * T;
        for (int dt = 0; dt < W; ++dt) {
            const int t = w + dt;
            float *z = out + ((size_t)r * W + dt) * D;
            if (t < 0 || t >= T)
                return -1;
            z[0] = yr[t];                                   /* target future y_t */
            for (int m = 0; m < d_y; ++m) {                 /* target past, eq. 7 */
                const int ti = t - 1 - m * tau;
                if (ti < 0)
                    return -1;
                z[1 + m] = yr[ti];
            }
            for (int m = 0; m < d_x; ++m) {                 /* source past at t-u */
                const int ti = t - u - m * tau;
                if (ti < 0)
                    return -1;
                z[1 + d_y + m] = xr[ti];
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------- distances */

/* |a - b| with the difference rounded to binary32 (mode 0) or kept exact in
 * double (mode 1, a diagnostic of the rounding choice only). */
static double absdiff(float a, float b, int mode)
{
    double d = (double)a - (double)b;
    if (mode == 0)
        d = (double)(float)d;
    return fabs(d);
}

/* max-norm distance between points p and q over coordinates [lo, hi); 0 if empty */
static double maxnorm(const float *p, const float *q, int lo, int hi, int mode)
{
    double m = 0.0;
    for (int c = lo; c < hi; ++c) {
        const double v = absdiff(p[c], q[c], mode);
        if (v > m)
            m = v;
    }
    return m;
}

/* Radius and the three strict counts of reference point i of one chunk, by
 * brute force over all j != i (O(N D)).  best: scratch of k doubles. */
static void point_stats(const float *pts, int N, int d_y, int d_x, int k, int mode, int i,
                        double *best, double *eps, int32_t *n_p, int32_t *n_tp, int32_t *n_ps)
{
    const int D = 1 + d_y + d_x;
    const float *pi = pts + (size_t)i * D;
    /* k smallest joint distances, kept sorted ascending */
    for (int s = 0; s < k; ++s)
        best[s] = INFINITY;
    for (int j = 0; j < N; ++j) {
        if (j == i)
            continue;
        const double d = maxnorm(pi, pts + (size_t)j * D, 0, D, mode);
        if (d < best[k - 1]) {
            int s = k - 1;
            while (s > 0 && best[s - 1] > d) {
                best[s] = best[s - 1];
                --s;
            }
            best[s] = d;
        }
    }
    const double e = best[k - 1];
    int32_t cp = 0, ctp = 0, cps = 0;
    for (int j = 0; j < N; ++j) {
        if (j == i)
            continue;
        const float *pj = pts + (size_t)j * D;
        if (maxnorm(pi, pj, 1, 1 + d_y, mode) < e)          /* P  */
            ++cp;
        if (maxnorm(pi, pj, 0, 1 + d_y, mode) < e)          /* TP */
            ++ctp;
        if (maxnorm(pi, pj, 1, D, mode) < e)                /* PS */
            ++cps;
    }
    *eps = e;
    *n_p = cp;
    *n_tp = ctp;
    *n_ps = cps;
}

/* Radius and the three strict counts for every point of one chunk.
 *   pts    float32 [N][D], D = 1 + d_y + d_x, coordinates ordered (T | P | S)
 *   eps    out [N]: distance to the k-th nearest neighbour in the joint space
 *   n_p, n_tp, n_ps  out [N]: #{ j != i : d_space(i, j) < eps_i } for the spaces
 *          P = target past, TP = target future + past, PS = target past + source past
 * Returns 0, or -1 if N <= k or k < 1. */
int ksg_counts(const float *pts, int N, int d_y, int d_x, int k, int mode,
               double *eps, int32_t *n_p, int32_t *n_tp, int32_t *n_ps)
{
    if (k < 1 || N <= k)
        return -1;
    double *best = (double *)malloc(sizeof(double) * (size_t)k);
    if (!best)
        return -1;
    for (int i = 0; i < N; ++i)
        point_stats(pts, N, d_y, d_x, k, mode, i, best, eps + i, n_p + i, n_tp + i, n_ps + i);
    free(best);
    return 0;
}

/* The same statistics for the listed reference points only: entry q of the
 * outputs belongs to point idx[q] (each O(N D), so single points of very large
 * chunks can be checked).  Returns 0, or -1 if N <= k, k < 1 or an index is
 * outside [0, N). */
int ksg_counts_points(const float *pts, int N, int d_y, int d_x, int k, int mode,
                      const int64_t *idx, int n_idx,
                      double *eps, int32_t *n_p, int32_t *n_tp, int32_t *n_ps)
{
    if (k < 1 || N <= k)
        return -1;
    for (int q = 0; q < n_idx; ++q)
        if (idx[q] < 0 || idx[q] >= N)
            return -1;
    double *best = (double *)malloc(sizeof(double) * (size_t)k);
    if (!best)
        return -1;
    for (int q = 0; q < n_idx; ++q)
        point_stats(pts, N, d_y, d_x, k, mode, (int)idx[q], best, eps + q, n_p + q, n_tp + q, n_ps + q);
    free(best);
    return 0;
}

/* ksg_counts with the reference points split over threads: thread t takes the
 * contiguous range of points [t N / n, (t+1) N / n).  Every point's statistics
 * come from the same brute-force loop, so the result is that of ksg_counts. */
typedef struct {
    const float *pts;
    int N, d_y, d_x, k, mode, i0, i1;
    double *eps;
    int32_t *n_p, *n_tp, *n_ps;
    int status;
} split_t;

static void *split_worker(void *arg)
{
    split_t *a = (split_t *)arg;
    double *best = (double *)malloc(sizeof(double) * (size_t)a->k);
    if (!best) {
        a->status = -1;
        return NULL;
    }
    for (int i = a->i0; i < a->i1; ++i)
        point_stats(a->pts, a->N, a->d_y, a->d_x, a->k, a->mode, i, best, a->eps + i, a->n_p + i,
                    a->n_tp + i, a->n_ps + i);
    free(best);
    a->status = 0;
    return NULL;
}

int ksg_counts_split(const float *pts, int N, int d_y, int d_x, int k, int mode, int n_threads,
                     double *eps, int32_t *n_p, int32_t *n_tp, int32_t *n_ps)
{
    if (k < 1 || N <= k)
        return -1;
    if (n_threads <= 0)
        n_threads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (n_threads > N)
        n_threads = N;
    split_t *parts = (split_t *)calloc((size_t)n_threads, sizeof(split_t));
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    if (!parts || !th) {
        free(parts);
        free(th);
        return -1;
    }
    for (int t = 0; t < n_threads; ++t) {
        split_t *a = &parts[t];
        a->pts = pts; a->N = N; a->d_y = d_y; a->d_x = d_x; a->k = k; a->mode = mode;
        a->i0 = (int)((int64_t)t * N / n_threads);
        a->i1 = (int)((int64_t)(t + 1) * N / n_threads);
        a->eps = eps; a->n_p = n_p; a->n_tp = n_tp; a->n_ps = n_ps;
        a->status = -1;
        pthread_create(&th[t], NULL, split_worker, a);
    }
    int bad = 0;
    for (int t = 0; t < n_threads; ++t) {
        pthread_join(th[t], NULL);
        bad |= parts[t].status != 0;
    }
    free(parts);
    free(th);
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------- estimator */

/* psi(n) for integer n >= 1: psi(1) = -gamma, psi(n+1) = psi(n) + 1/n,
 * accumulated in long double. */
double ksg_digamma_int(int n)
{
    const long double euler_gamma = 0.57721566490153286060651209008240243L;
    long double h = 0.0L;
    for (int m = 1; m < n; ++m)
        h += 1.0L / (long double)m;
    return (double)(h - euler_gamma);
}

/* eq. 9 / 10: psi(k) + mean_i [ psi(n_P+1) - psi(n_TP+1) - psi(n_PS+1) ] */
double ksg_te_from_counts(const int32_t *n_p, const int32_t *n_tp, const int32_t *n_ps,
                          int N, int k)
{
    int nmax = 0;
    for (int i = 0; i < N; ++i) {
        if (n_p[i] > nmax) nmax = n_p[i];
        if (n_tp[i] > nmax) nmax = n_tp[i];
        if (n_ps[i] > nmax) nmax = n_ps[i];
    }
    /* psi(n+1) for n = 0..nmax, by the recurrence in long double */
    const long double euler_gamma = 0.57721566490153286060651209008240243L;
    long double *psi1 = (long double *)malloc(sizeof(long double) * ((size_t)nmax + 1));
    if (!psi1)
        return NAN;
    psi1[0] = -euler_gamma;
    for (int n = 1; n <= nmax; ++n)
        psi1[n] = psi1[n - 1] + 1.0L / (long double)n;
    long double acc = 0.0L;
    for (int i = 0; i < N; ++i)
        acc += psi1[n_p[i]] - psi1[n_tp[i]] - psi1[n_ps[i]];
    free(psi1);
    return ksg_digamma_int(k) + (double)(acc / (long double)N);
}

/* Local TE of each pooled point (the summand of eq. 9 with psi(k) added, the
 * per-event quantity of eq. 17 estimated on the ensemble PDF): its mean over the
 * points is eq. 9's estimate (eq. 18).  Harmonic numbers in long double; gamma
 * cancels since it enters twice with each sign. */
void ksg_local_from_counts(const int32_t *n_p, const int32_t *n_tp, const int32_t *n_ps, int N, int k,
                           double *lte)
{
    for (int i = 0; i < N; ++i) {
        long double h = 0.0L;
        for (int m = 1; m < k; ++m)
            h += 1.0L / (long double)m;
        for (int m = 1; m <= n_p[i]; ++m)
            h += 1.0L / (long double)m;
        for (int m = 1; m <= n_tp[i]; ++m)
            h -= 1.0L / (long double)m;
        for (int m = 1; m <= n_ps[i]; ++m)
            h -= 1.0L / (long double)m;
        lte[i] = (double)h;
    }
}

/* p = #{ s : te_surr[s] >= te_orig } / S  (NaN when S == 0) */
double ksg_p_value(double te_orig, const double *te_surr, int S)
{
    if (S <= 0)
        return NAN;
    int c = 0;
    for (int s = 0; s < S; ++s)
        if (te_surr[s] >= te_orig)
            ++c;
    return (double)c / (double)S;
}

/* ------------------------------------------------- whole estimates, threaded */

typedef struct {
    const float *x, *y;
    int R, T, d_y, d_x, tau, u, k, mode;
    int n_jobs;
    const int32_t *pair, *w, *W, *Rc, *perm_row; /* perm_row: -1 = original */
    const int32_t *perms;                          /* [n_perm_rows][R] */
    double *te;
    int32_t *status;
    int next;
    pthread_mutex_t lock;
} batch_t;

static void *batch_worker(void *arg)
{
    batch_t *b = (batch_t *)arg;
    for (;;) {
        pthread_mutex_lock(&b->lock);
        const int j = b->next++;
        pthread_mutex_unlock(&b->lock);
        if (j >= b->n_jobs)
            break;
        const int N = b->Rc[j] * b->W[j];
        const int D = 1 + b->d_y + b->d_x;
        float *pts = (float *)malloc(sizeof(float) * (size_t)N * D);
        double *eps = (double *)malloc(sizeof(double) * (size_t)N);
        int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)N);
        int st = -1;
        if (pts && eps && cnt) {
            const size_t off = (size_t)b->pair[j] * b->R * b->T;
            const int32_t *sp = b->perm_row[j] >= 0 ? b->perms + (size_t)b->perm_row[j] * b->R : NULL;
            st = ksg_embed(b->x + off, b->y + off, b->R, b->T, b->d_y, b->d_x, b->tau, b->u,
                           b->w[j], b->W[j], b->Rc[j], sp, NULL, pts);
            if (st == 0)
                st = ksg_counts(pts, N, b->d_y, b->d_x, b->k, b->mode, eps,
                                cnt, cnt + N, cnt + 2 * (size_t)N);
            if (st == 0)
                b->te[j] = ksg_te_from_counts(cnt, cnt + N, cnt + 2 * (size_t)N, N, b->k);
        }
        b->status[j] = st;
        free(pts);
        free(eps);
        free(cnt);
    }
    return NULL;
}

/* TE of n_jobs independent chunks, spread over n_threads threads (0 = all online
 * cores).  Job j pools repetitions r < Rc[j] over the window [w[j], w[j]+W[j]) of
 * pair pair[j]; perm_row[j] >= 0 selects the source permutation perms[perm_row[j]][:].
 * Returns the number of failed jobs (their te is left untouched). */
int ksg_te_batch(const float *x, const float *y, int R, int T,
                 int d_y, int d_x, int tau, int u, int k, int mode,
                 int n_jobs, const int32_t *pair, const int32_t *w, const int32_t *W,
                 const int32_t *Rc, const int32_t *perm_row, const int32_t *perms,
                 int n_threads, double *te)
{
    batch_t b;
    memset(&b, 0, sizeof b);
    b.x = x; b.y = y; b.R = R; b.T = T; b.d_y = d_y; b.d_x = d_x; b.tau = tau; b.u = u;
    b.k = k; b.mode = mode; b.n_jobs = n_jobs; b.pair = pair; b.w = w; b.W = W; b.Rc = Rc;
    b.perm_row = perm_row; b.perms = perms; b.te = te;
    b.status = (int32_t *)calloc((size_t)(n_jobs > 0 ? n_jobs : 1), sizeof(int32_t));
    pthread_mutex_init(&b.lock, NULL);
    if (n_threads <= 0)
        n_threads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (n_threads > n_jobs)
        n_threads = n_jobs > 0 ? n_jobs : 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    for (int t = 0; t < n_threads; ++t)
        pthread_create(&th[t], NULL, batch_worker, &b);
    for (int t = 0; t < n_threads; ++t)
        pthread_join(th[t], NULL);
    int bad = 0;
    for (int j = 0; j < n_jobs; ++j)
        bad += b.status[j] != 0;
    free(th);
    free(b.status);
    pthread_mutex_destroy(&b.lock);
    return bad;
}

/* Neighbour statistics for several pre-embedded chunks in parallel: chunk c is
 * float32 [N_c][D] at pts + off[c]*D, results at eps + off[c] and cnt[3][off[c]..]. */
typedef struct {
    const float *pts;
    const int64_t *off;
    int n_chunks, d_y, d_x, k, mode;
    int64_t total;
    double *eps;
    int32_t *cnt;
    int32_t *status;
    int next;
    pthread_mutex_t lock;
} cbatch_t;

static void *cbatch_worker(void *arg)
{
    cbatch_t *b = (cbatch_t *)arg;
    const int D = 1 + b->d_y + b->d_x;
    for (;;) {
        pthread_mutex_lock(&b->lock);
        const int c = b->next++;
        pthread_mutex_unlock(&b->lock);
        if (c >= b->n_chunks)
            break;
        const int64_t o = b->off[c];
        const int N = (int)(b->off[c + 1] - o);
        b->status[c] = ksg_counts(b->pts + o * D, N, b->d_y, b->d_x, b->k, b->mode, b->eps + o,
                                  b->cnt + o, b->cnt + b->total + o, b->cnt + 2 * b->total + o);
    }
    return NULL;
}

int ksg_counts_batch(const float *pts, const int64_t *off, int n_chunks, int d_y, int d_x, int k,
                     int mode, int n_threads, double *eps, int32_t *cnt)
{
    cbatch_t b;
    memset(&b, 0, sizeof b);
    b.pts = pts; b.off = off; b.n_chunks = n_chunks; b.d_y = d_y; b.d_x = d_x; b.k = k;
    b.mode = mode; b.total = off[n_chunks]; b.eps = eps; b.cnt = cnt;
    b.status = (int32_t *)calloc((size_t)(n_chunks > 0 ? n_chunks : 1), sizeof(int32_t));
    pthread_mutex_init(&b.lock, NULL);
    if (n_threads <= 0)
        n_threads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (n_threads > n_chunks)
        n_threads = n_chunks > 0 ? n_chunks : 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    for (int t = 0; t < n_threads; ++t)
        pthread_create(&th[t], NULL, cbatch_worker, &b);
    for (int t = 0; t < n_threads; ++t)
        pthread_join(th[t], NULL);
    int bad = 0;
    for (int c = 0; c < n_chunks; ++c)
        bad += b.status[c] != 0;
    free(th);
    free(b.status);
    pthread_mutex_destroy(&b.lock);
    return bad;
}
