/* CPU check of the oracle under AddressSanitizer / UndefinedBehaviorSanitizer,
 * built with gcc by tests/test_host_sanitizers.py:
 *   oracle_checks <in> <out>
 * <in>:  int64 cases; per case int32 kind (0 auto, 1 cross), int32 m, tau,
 *        norm, theiler, lmin, vmin, wmin, float eps, int64 na, nb (nb = 0 for
 *        auto), then na (and nb) float32 points.
 * <out>: per case the three histograms (uint64, exact length) and the 15
 *        measures (FP64) of the oracle, with one thread and with four. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t rqa_oracle_n_vectors(int64_t n_points, int m, int tau);
int rqa_oracle_histograms(const float *s, int64_t n_points, int m, int tau, float eps, int norm,
                          int theiler, uint64_t *diag, uint64_t *vert, uint64_t *white,
                          int threads);
int rqa_oracle_cross_histograms(const float *a, int64_t na_points, const float *b,
                                int64_t nb_points, int m, int tau, float eps, int norm,
                                int theiler, uint64_t *diag, uint64_t *vert, uint64_t *white,
                                int threads);
int rqa_oracle_measures(const uint64_t *diag, const uint64_t *vert, const uint64_t *white,
                        int64_t n, int theiler, int lmin, int vmin, int wmin, double *out);
int rqa_oracle_rect_measures(const uint64_t *diag, const uint64_t *vert, const uint64_t *white,
                             int64_t n_rows, int64_t n_cols, int theiler, int lmin, int vmin,
                             int wmin, double *out);

static int fail(const char *what)
{
    fprintf(stderr, "oracle_checks: %s\n", what);
    return 1;
}

int main(int argc, char **argv)
{
    FILE *f, *g;
    int64_t cases, c;
    if (argc < 3)
        return fail("usage: oracle_checks <in> <out>");
    f = fopen(argv[1], "rb");
    g = fopen(argv[2], "wb");
    if (!f || !g)
        return fail("cannot open files");
    if (fread(&cases, sizeof cases, 1, f) != 1)
        return fail("short input");
    for (c = 0; c < cases; ++c) {
        int32_t hdr[8];
        float eps;
        int64_t na, nb, len, n_rows, n_cols;
        float *a, *b = NULL;
        int t;
        if (fread(hdr, sizeof hdr, 1, f) != 1 || fread(&eps, sizeof eps, 1, f) != 1 ||
            fread(&na, sizeof na, 1, f) != 1 || fread(&nb, sizeof nb, 1, f) != 1)
            return fail("bad case header");
        a = malloc(sizeof(float) * (size_t)na);
        if (!a || fread(a, sizeof(float), (size_t)na, f) != (size_t)na)
            return fail("short series");
        if (hdr[0] == 1) {
            b = malloc(sizeof(float) * (size_t)nb);
            if (!b || fread(b, sizeof(float), (size_t)nb, f) != (size_t)nb)
                return fail("short second series");
        }
        n_rows = rqa_oracle_n_vectors(na, hdr[1], hdr[2]);
        n_cols = hdr[0] == 1 ? rqa_oracle_n_vectors(nb, hdr[1], hdr[2]) : n_rows;
        len = (n_rows > n_cols ? n_rows : n_cols) + 1;
        for (t = 1; t <= 4; t += 3) {
            /* exact-size buffers, so that a write past len entries is caught */
            uint64_t *d = malloc(sizeof(uint64_t) * (size_t)len);
            uint64_t *v = malloc(sizeof(uint64_t) * (size_t)len);
            uint64_t *w = malloc(sizeof(uint64_t) * (size_t)len);
            double meas[15];
            int rc;
            if (!d || !v || !w)
                return fail("out of memory");
            if (hdr[0] == 1)
                rc = rqa_oracle_cross_histograms(a, na, b, nb, hdr[1], hdr[2], eps, hdr[3], hdr[4],
                                                 d, v, w, t);
            else
                rc = rqa_oracle_histograms(a, na, hdr[1], hdr[2], eps, hdr[3], hdr[4], d, v, w, t);
            if (rc != 0)
                return fail("oracle rejected a case");
            if (hdr[0] == 1)
                rc = rqa_oracle_rect_measures(d, v, w, n_rows, n_cols, hdr[4], hdr[5], hdr[6],
                                              hdr[7], meas);
            else
                rc = rqa_oracle_measures(d, v, w, n_rows, hdr[4], hdr[5], hdr[6], hdr[7], meas);
            if (rc != 0)
                return fail("measures rejected a case");
            fwrite(d, sizeof(uint64_t), (size_t)len, g);
            fwrite(v, sizeof(uint64_t), (size_t)len, g);
            fwrite(w, sizeof(uint64_t), (size_t)len, g);
            fwrite(meas, sizeof(double), 15, g);
            free(d);
            free(v);
            free(w);
        }
        free(a);
        free(b);
    }
    fclose(f);
    fclose(g);
    return 0;
}
