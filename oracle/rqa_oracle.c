/*
 * rqa_oracle.c -- plain CPU reference for recurrence quantification analysis.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header or table with the
 * HIP implementation.
 *
 * What it computes (the plain definition, Sect. 2 "Basic Concepts of RQA" and
 * the parameter list of Sect. 7.2):
 *
 *   embedding   x_i = (s[i], s[i+tau], ..., s[i+(m-1)tau]),  i = 0..n-1,
 *               n = N - (m-1)tau                      (time-delay embedding)
 *   similarity  d_k = s[i+k tau] - s[j+k tau]  in FP32, k ascending, no FMA;
 *               L1:  a = |d_0| + |d_1| + ... (left to right)     R = a <= eps
 *               L2:  a = d_0 d_0 + d_1 d_1 + ... (left to right) R = a <= fl32(eps*eps)
 *               Linf a = max_k |d_k|                             R = a <= eps
 *               (fixed radius neighbourhood; the L2 form compares the squared
 *               sum so no square root is rounded)
 *   Theiler     R_ij = 0 when |i-j| < w
 *   lines       diagonal lines (runs of 1 along i-j = const), vertical lines
 *               (runs of 1 down a column) and white vertical lines (runs of 0
 *               down a column) of the whole n x n matrix, both triangles,
 *               including runs that touch the matrix border (Sect. 2 list of
 *               the three line types; Sect. 4.2 operators II and III inspect
 *               one diagonal / one column each).
 *
 * The diagonal pass walks the diagonals k = w..n-1 of the upper triangle one
 * cell at a time and counts every run twice (the matrix is exactly symmetric
 * because |a-b| = |b-a| in IEEE arithmetic, so diagonal -k repeats diagonal k);
 * the main diagonal (only present when w = 0) is counted once.  The column pass
 * walks every column j over all rows i = 0..n-1 and evaluates the predicate
 * for every cell, the way a sequential on-the-fly tool would.  Memory is O(n).
 *
 * Cross recurrence (the cRQA discussion of the related work, and Sect. 4.2,
 * where a non-symmetric matrix has 2N-1 diagonals): rows are the delay vectors
 * of a series a, columns those of a series b, same m, tau, norm and radius; the
 * matrix is n_a x n_b and not symmetric, so every diagonal k = j - i from
 * -(n_a-1) to n_b-1 is walked and each run counted once; columns run over all
 * n_a rows.  The optional Theiler window masks |i-j| < w by index.
 *
 * Given matrix: the same three histograms of a caller-supplied bit matrix
 * (row-major, bit b of 64-bit word c of row i = column 64c+b).
 *
 * Build: gcc -O2 -ffp-contract=off (no -ffast-math); FP32 denormals are kept.
 * Measures (Sect. 8.1, Tab. 3 names; definitions are the standard ones) are
 * computed in FP64 from the integer histograms.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_L1 1
#define ORACLE_L2 2
#define ORACLE_LINF 3

/* Recurrence predicate for the vector pair (i, j): one FP32 operation at a time
 * in ascending coordinate order. */
static int oracle_recurrent(const float *s, int64_t i, int64_t j, int m, int tau,
                            int norm, float eps, float eps_sq)
{
    int k;
    if (norm == ORACLE_L1) {
        float a = fabsf(s[i] - s[j]);
        for (k = 1; k < m; ++k) {
            float d = s[i + (int64_t)k * tau] - s[j + (int64_t)k * tau];
            a = a + fabsf(d);
        }
        return a <= eps;
    }
    if (norm == ORACLE_L2) {
        float d = s[i] - s[j];
        float a = d * d;
        for (k = 1; k < m; ++k) {
            float e = s[i + (int64_t)k * tau] - s[j + (int64_t)k * tau];
            float sq = e * e;
            a = a + sq;
        }
        return a <= eps_sq;
    }
    {
        float a = fabsf(s[i] - s[j]);
        for (k = 1; k < m; ++k) {
            float b = fabsf(s[i + (int64_t)k * tau] - s[j + (int64_t)k * tau]);
            if (b > a)
                a = b;
        }
        return a <= eps;
    }
}

/* Masked matrix element: zero inside the Theiler band |i-j| < w. */
static int oracle_cell(const float *s, int64_t i, int64_t j, int m, int tau, int norm,
                       float eps, float eps_sq, int64_t w)
{
    int64_t gap = i > j ? i - j : j - i;
    if (gap < w)
        return 0;
    return oracle_recurrent(s, i, j, m, tau, norm, eps, eps_sq);
}

int64_t rqa_oracle_n_vectors(int64_t n_points, int m, int tau)
{
    return n_points - (int64_t)(m - 1) * tau;
}

/* Histograms of the whole masked matrix.  diag, vert and white each hold n+1
 * entries, indexed by line length (entry 0 stays 0); the callee zeroes them.
 * Returns 0, or -1 for invalid arguments. */
int rqa_oracle_histograms(const float *s, int64_t n_points, int m, int tau, float eps,
                          int norm, int theiler, uint64_t *diag, uint64_t *vert,
                          uint64_t *white, int threads)
{
    int64_t n, k, j;
    float eps_sq;
    int nt;
    if (!s || !diag || !vert || !white || m < 1 || tau < 1 || theiler < 0 ||
        norm < 1 || norm > 3 || !(eps >= 0.0f) || isinf(eps))
        return -1;
    n = rqa_oracle_n_vectors(n_points, m, tau);
    if (n < 1)
        return -1;
    eps_sq = eps * eps;
    memset(diag, 0, sizeof(uint64_t) * (size_t)(n + 1));
    memset(vert, 0, sizeof(uint64_t) * (size_t)(n + 1));
    memset(white, 0, sizeof(uint64_t) * (size_t)(n + 1));

#ifdef _OPENMP
    nt = threads > 0 ? threads : omp_get_max_threads();
#else
    nt = 1;
    (void)threads;
#endif

    /* ---- diagonal lines (operator II): one diagonal at a time ---- */
#pragma omp parallel num_threads(nt)
    {
        uint64_t *ld = (uint64_t *)calloc((size_t)(n + 1), sizeof(uint64_t));
        uint64_t *lv = (uint64_t *)calloc((size_t)(n + 1), sizeof(uint64_t));
        uint64_t *lw = (uint64_t *)calloc((size_t)(n + 1), sizeof(uint64_t));
#pragma omp for schedule(dynamic, 16)
        for (k = theiler; k < n; ++k) {
            uint64_t weight = (k == 0) ? 1 : 2; /* diagonal -k mirrors diagonal k */
            int64_t run = 0, t;
            for (t = 0; t + k < n; ++t) {
                if (oracle_cell(s, t, t + k, m, tau, norm, eps, eps_sq, theiler)) {
                    run += 1;
                } else if (run > 0) {
                    ld[run] += weight;
                    run = 0;
                }
            }
            if (run > 0)
                ld[run] += weight;
        }

        /* ---- vertical and white vertical lines (operator III): one column at a time ---- */
#pragma omp for schedule(dynamic, 16)
        for (j = 0; j < n; ++j) {
            int64_t black = 0, blank = 0, i;
            for (i = 0; i < n; ++i) {
                if (oracle_cell(s, i, j, m, tau, norm, eps, eps_sq, theiler)) {
                    if (blank > 0) {
                        lw[blank] += 1;
                        blank = 0;
                    }
                    black += 1;
                } else {
                    if (black > 0) {
                        lv[black] += 1;
                        black = 0;
                    }
                    blank += 1;
                }
            }
            if (black > 0)
                lv[black] += 1;
            if (blank > 0)
                lw[blank] += 1;
        }

#pragma omp critical
        {
            int64_t l;
            for (l = 0; l <= n; ++l) {
                diag[l] += ld[l];
                vert[l] += lv[l];
                white[l] += lw[l];
            }
        }
        free(ld);
        free(lv);
        free(lw);
    }
    return 0;
}

/* Predicate for row vector i of series a and column vector j of series b, the
 * same operation sequence as oracle_recurrent with s[i + k tau] taken from a and
 * s[j + k tau] from b. */
static int oracle_cross_recurrent(const float *a, int64_t i, const float *b, int64_t j, int m,
                                  int tau, int norm, float eps, float eps_sq)
{
    int k;
    if (norm == ORACLE_L1) {
        float acc = fabsf(a[i] - b[j]);
        for (k = 1; k < m; ++k) {
            float d = a[i + (int64_t)k * tau] - b[j + (int64_t)k * tau];
            acc = acc + fabsf(d);
        }
        return acc <= eps;
    }
    if (norm == ORACLE_L2) {
        float d = a[i] - b[j];
        float acc = d * d;
        for (k = 1; k < m; ++k) {
            float e = a[i + (int64_t)k * tau] - b[j + (int64_t)k * tau];
            float sq = e * e;
            acc = acc + sq;
        }
        return acc <= eps_sq;
    }
    {
        float acc = fabsf(a[i] - b[j]);
        for (k = 1; k < m; ++k) {
            float t = fabsf(a[i + (int64_t)k * tau] - b[j + (int64_t)k * tau]);
            if (t > acc)
                acc = t;
        }
        return acc <= eps;
    }
}

/* Cell (i, j) of one of the two non-symmetric matrices: the cross recurrence
 * matrix of (a, b), or a given bit matrix. */
typedef struct {
    const float *a, *b;
    int m, tau, norm;
    float eps, eps_sq;
    const uint64_t *bits;   /* non-NULL: given matrix */
    int64_t words;          /* 64-bit words per row of the given matrix */
    int64_t w;              /* Theiler window */
} oracle_rect;

static int oracle_rect_cell(const oracle_rect *r, int64_t i, int64_t j)
{
    int64_t gap = i > j ? i - j : j - i;
    if (gap < r->w)
        return 0;
    if (r->bits)
        return (int)((r->bits[i * r->words + (j >> 6)] >> (j & 63)) & 1u);
    return oracle_cross_recurrent(r->a, i, r->b, j, r->m, r->tau, r->norm, r->eps, r->eps_sq);
}

/* Lines of an n_rows x n_cols matrix: every diagonal k = j - i once, every
 * column over all rows.  Histograms hold max(n_rows, n_cols)+1 entries. */
static void oracle_rect_histograms(const oracle_rect *r, int64_t n_rows, int64_t n_cols,
                                   uint64_t *diag, uint64_t *vert, uint64_t *white, int nt)
{
    int64_t len = (n_rows > n_cols ? n_rows : n_cols) + 1, k, j;
    memset(diag, 0, sizeof(uint64_t) * (size_t)len);
    memset(vert, 0, sizeof(uint64_t) * (size_t)len);
    memset(white, 0, sizeof(uint64_t) * (size_t)len);
#pragma omp parallel num_threads(nt)
    {
        uint64_t *ld = (uint64_t *)calloc((size_t)len, sizeof(uint64_t));
        uint64_t *lv = (uint64_t *)calloc((size_t)len, sizeof(uint64_t));
        uint64_t *lw = (uint64_t *)calloc((size_t)len, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 16)
        for (k = -(n_rows - 1); k < n_cols; ++k) {
            int64_t run = 0, t = k < 0 ? -k : 0;
            for (; t < n_rows && t + k < n_cols; ++t) {
                if (oracle_rect_cell(r, t, t + k)) {
                    run += 1;
                } else if (run > 0) {
                    ld[run] += 1;
                    run = 0;
                }
            }
            if (run > 0)
                ld[run] += 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (j = 0; j < n_cols; ++j) {
            int64_t black = 0, blank = 0, i;
            for (i = 0; i < n_rows; ++i) {
                if (oracle_rect_cell(r, i, j)) {
                    if (blank > 0) {
                        lw[blank] += 1;
                        blank = 0;
                    }
                    black += 1;
                } else {
                    if (black > 0) {
                        lv[black] += 1;
                        black = 0;
                    }
                    blank += 1;
                }
            }
            if (black > 0)
                lv[black] += 1;
            if (blank > 0)
                lw[blank] += 1;
        }
#pragma omp critical
        {
            int64_t l;
            for (l = 0; l < len; ++l) {
                diag[l] += ld[l];
                vert[l] += lv[l];
                white[l] += lw[l];
            }
        }
        free(ld);
        free(lv);
        free(lw);
    }
}

static int oracle_threads(int threads)
{
#ifdef _OPENMP
    return threads > 0 ? threads : omp_get_max_threads();
#else
    (void)threads;
    return 1;
#endif
}

/* Cross recurrence histograms of series a (rows) against series b (columns);
 * each array holds max(n_a, n_b)+1 entries.  Returns 0, or -1 for invalid
 * arguments. */
int rqa_oracle_cross_histograms(const float *a, int64_t na_points, const float *b,
                                int64_t nb_points, int m, int tau, float eps, int norm,
                                int theiler, uint64_t *diag, uint64_t *vert, uint64_t *white,
                                int threads)
{
    oracle_rect r;
    int64_t na, nb;
    if (!a || !b || !diag || !vert || !white || m < 1 || tau < 1 || theiler < 0 ||
        norm < 1 || norm > 3 || !(eps >= 0.0f) || isinf(eps))
        return -1;
    na = rqa_oracle_n_vectors(na_points, m, tau);
    nb = rqa_oracle_n_vectors(nb_points, m, tau);
    if (na < 1 || nb < 1)
        return -1;
    r.a = a;
    r.b = b;
    r.m = m;
    r.tau = tau;
    r.norm = norm;
    r.eps = eps;
    r.eps_sq = eps * eps;
    r.bits = NULL;
    r.words = 0;
    r.w = theiler;
    oracle_rect_histograms(&r, na, nb, diag, vert, white, oracle_threads(threads));
    return 0;
}

/* Histograms of a given n_rows x n_cols bit matrix (row-major 64-bit words,
 * `words` per row, bit b of word c = column 64c+b); cells inside the Theiler
 * band |i-j| < theiler count as 0.  Arrays hold max(n_rows, n_cols)+1 entries. */
int rqa_oracle_matrix_histograms(const uint64_t *bits, int64_t n_rows, int64_t n_cols,
                                 int64_t words, int theiler, uint64_t *diag, uint64_t *vert,
                                 uint64_t *white, int threads)
{
    oracle_rect r;
    if (!bits || !diag || !vert || !white || n_rows < 1 || n_cols < 1 || theiler < 0 ||
        words < (n_cols + 63) / 64)
        return -1;
    memset(&r, 0, sizeof r);
    r.bits = bits;
    r.words = words;
    r.w = theiler;
    oracle_rect_histograms(&r, n_rows, n_cols, diag, vert, white, oracle_threads(threads));
    return 0;
}

/* Recurrence plot (Sect. 4 and the workflow classes of Sect. 7): the
 * masked matrix packed row-major, `words` 64-bit words per row, bit b of word c
 * of row i = cell (i, 64c+b); bits past the last column are 0.  b == NULL: the
 * n x n matrix of series a; otherwise the cross matrix of a (rows) and b
 * (columns).  Returns 0, or -1 for invalid arguments. */
int rqa_oracle_plot(const float *a, int64_t na_points, const float *b, int64_t nb_points, int m,
                    int tau, float eps, int norm, int theiler, uint64_t *bits, int64_t words)
{
    oracle_rect r;
    int64_t na, nb, i, j;
    if (!a || !bits || m < 1 || tau < 1 || theiler < 0 || norm < 1 || norm > 3 ||
        !(eps >= 0.0f) || isinf(eps))
        return -1;
    na = rqa_oracle_n_vectors(na_points, m, tau);
    nb = b ? rqa_oracle_n_vectors(nb_points, m, tau) : na;
    if (na < 1 || nb < 1 || words < (nb + 63) / 64)
        return -1;
    r.a = a;
    r.b = b ? b : a;
    r.m = m;
    r.tau = tau;
    r.norm = norm;
    r.eps = eps;
    r.eps_sq = eps * eps;
    r.bits = NULL;
    r.words = 0;
    r.w = theiler;
    memset(bits, 0, sizeof(uint64_t) * (size_t)(na * words));
    for (i = 0; i < na; ++i)
        for (j = 0; j < nb; ++j)
            if (oracle_rect_cell(&r, i, j))
                bits[i * words + (j >> 6)] |= (uint64_t)1 << (j & 63);
    return 0;
}

/* Measure vector layout (all FP64):
 *  0 RR  1 DET  2 L  3 Lmax  4 DIV  5 L_entr  6 LAM  7 TT  8 Vmax  9 V_entr
 * 10 W  11 Wmax 12 W_entr 13 N_rec 14 n */
#define ORACLE_NMEAS 15

/* Cells of an n_rows x n_cols matrix outside the band |i-j| < w, counted row by
 * row. */
static double oracle_rect_cells_outside_band(int64_t n_rows, int64_t n_cols, int64_t w)
{
    double band = 0.0;
    int64_t i;
    if (w <= 0)
        return (double)n_rows * (double)n_cols;
    for (i = 0; i < n_rows; ++i) {
        int64_t lo = i - (w - 1), hi = i + (w - 1);
        if (lo < 0)
            lo = 0;
        if (hi > n_cols - 1)
            hi = n_cols - 1;
        if (hi >= lo)
            band += (double)(hi - lo + 1);
    }
    return (double)n_rows * (double)n_cols - band;
}

/* Cells outside the Theiler band: n^2 minus the band |i-j| < w. */
static double oracle_cells_outside_band(int64_t n, int64_t w)
{
    double band = 0.0;
    int64_t k;
    if (w <= 0)
        return (double)n * (double)n;
    band = (double)n; /* main diagonal */
    for (k = 1; k < w && k < n; ++k)
        band += 2.0 * (double)(n - k);
    return (double)n * (double)n - band;
}

/* sum over l >= from of l^p * h[l], p in {0, 1} (ascending l) */
static double oracle_sum(const uint64_t *h, int64_t n, int64_t from, int p)
{
    double acc = 0.0;
    int64_t l;
    for (l = from < 1 ? 1 : from; l <= n; ++l)
        acc += (p ? (double)l : 1.0) * (double)h[l];
    return acc;
}

static double oracle_longest(const uint64_t *h, int64_t n)
{
    int64_t l;
    for (l = n; l >= 1; --l)
        if (h[l] > 0)
            return (double)l;
    return 0.0;
}

/* Shannon entropy (natural log) of the line-length distribution over l >= from,
 * normalised by the number of such lines; empty classes are skipped.  The
 * paper fixes no summation order, so the terms -p ln p are added in ascending l
 * with Neumaier's compensated summation (the improved Kahan-Babuska sum): the
 * result is the sum of the computed terms to within a few ulps however many
 * classes there are (a plain running sum drifts by ~1e-11 relative over the
 * ~2.3e5 classes of a long, almost periodic series). */
static double oracle_entropy(const uint64_t *h, int64_t n, int64_t from)
{
    double total = oracle_sum(h, n, from, 0), sum = 0.0, comp = 0.0;
    int64_t l;
    if (total == 0.0)
        return NAN;
    for (l = from < 1 ? 1 : from; l <= n; ++l) {
        if (h[l] > 0) {
            double p = (double)h[l] / total;
            double term = -(p * log(p));
            double t = sum + term;
            if (fabs(sum) >= fabs(term))
                comp += (sum - t) + term;
            else
                comp += (term - t) + sum;
            sum = t;
        }
    }
    return sum + comp;
}

/* Measures from histograms of `n` entries past index 0 over `cells` matrix
 * cells outside the band; out[14] = n_report. */
static void oracle_measures_core(const uint64_t *diag, const uint64_t *vert,
                                 const uint64_t *white, int64_t n, double cells, int lmin,
                                 int vmin, int wmin, double n_report, double *out)
{
    double n_rec, det_num, lines_l, lam_num, v_all, lines_v, w_num, lines_w, lmax;
    n_rec = oracle_sum(diag, n, 1, 1);
    det_num = oracle_sum(diag, n, lmin, 1);
    lines_l = oracle_sum(diag, n, lmin, 0);
    v_all = oracle_sum(vert, n, 1, 1);
    lam_num = oracle_sum(vert, n, vmin, 1);
    lines_v = oracle_sum(vert, n, vmin, 0);
    w_num = oracle_sum(white, n, wmin, 1);
    lines_w = oracle_sum(white, n, wmin, 0);
    lmax = oracle_longest(diag, n);

    out[0] = n_rec / cells;                                  /* RR */
    out[1] = det_num / n_rec;                                /* DET */
    out[2] = det_num / lines_l;                              /* L */
    out[3] = lmax;                                           /* Lmax */
    out[4] = 1.0 / lmax;                                     /* DIV */
    out[5] = oracle_entropy(diag, n, lmin);                  /* L_entr */
    out[6] = lam_num / v_all;                                /* LAM */
    out[7] = lam_num / lines_v;                              /* TT */
    out[8] = oracle_longest(vert, n);                        /* Vmax */
    out[9] = oracle_entropy(vert, n, vmin);                  /* V_entr */
    out[10] = w_num / lines_w;                               /* W */
    out[11] = oracle_longest(white, n);                      /* Wmax */
    out[12] = oracle_entropy(white, n, wmin);                /* W_entr */
    out[13] = n_rec;
    out[14] = n_report;
    if (lmax == 0.0)
        out[4] = NAN;
}

int rqa_oracle_measures(const uint64_t *diag, const uint64_t *vert, const uint64_t *white,
                        int64_t n, int theiler, int lmin, int vmin, int wmin, double *out)
{
    if (!diag || !vert || !white || !out || n < 1)
        return -1;
    oracle_measures_core(diag, vert, white, n, oracle_cells_outside_band(n, theiler), lmin,
                         vmin, wmin, (double)n, out);
    return 0;
}

/* Measures of an n_rows x n_cols matrix (cross recurrence or a given matrix):
 * histograms of max(n_rows, n_cols)+1 entries; RR over the cells outside the
 * band; out[14] = n_rows. */
int rqa_oracle_rect_measures(const uint64_t *diag, const uint64_t *vert, const uint64_t *white,
                             int64_t n_rows, int64_t n_cols, int theiler, int lmin, int vmin,
                             int wmin, double *out)
{
    int64_t n = n_rows > n_cols ? n_rows : n_cols;
    if (!diag || !vert || !white || !out || n_rows < 1 || n_cols < 1)
        return -1;
    oracle_measures_core(diag, vert, white, n,
                         oracle_rect_cells_outside_band(n_rows, n_cols, theiler), lmin, vmin,
                         wmin, (double)n_rows, out);
    return 0;
}
