// Host-side RQA measures in FP64 from the integer line-length histograms.
//
// Definitions: the measures listed in Tab. 3 (RR, DET, L, Lmax, DIV, L_entr,
// LAM, TT, Vmax, V_entr) plus the white-vertical analogues (W, Wmax, W_entr),
// derived from the frequency distributions of the three line types (Sect. 2).
// Sums run over ascending line length; empty denominators give NaN.
#include <cmath>
#include <limits>

#include "rqa_internal.h"

namespace rqa {

namespace {

struct Moments {
    double count = 0.0;   // number of lines with length >= floor
    double mass = 0.0;    // sum of their lengths
};

Moments moments(const uint64_t *h, int64_t n, int64_t floor_len) {
    Moments mo;
    for (int64_t l = floor_len < 1 ? 1 : floor_len; l <= n; ++l) {
        if (h[l] == 0) continue;
        const double c = static_cast<double>(h[l]);
        mo.count += c;
        mo.mass += c * static_cast<double>(l);
    }
    return mo;
}

double longest(const uint64_t *h, int64_t n) {
    for (int64_t l = n; l >= 1; --l)
        if (h[l] != 0) return static_cast<double>(l);
    return 0.0;
}

// Shannon entropy (natural log) of the distribution of lines of length >= floor.
double entropy(const uint64_t *h, int64_t n, int64_t floor_len, double count) {
    if (count == 0.0) return std::numeric_limits<double>::quiet_NaN();
    double e = 0.0;
    for (int64_t l = floor_len < 1 ? 1 : floor_len; l <= n; ++l) {
        if (h[l] == 0) continue;
        const double p = static_cast<double>(h[l]) / count;
        e -= p * std::log(p);
    }
    return e;
}

double ratio(double a, double b) {
    return b == 0.0 ? std::numeric_limits<double>::quiet_NaN() : a / b;
}

// Cells of the n x n matrix outside the Theiler band |i-j| < w.
double cells_outside_band(int64_t n, int64_t w) {
    const double nn = static_cast<double>(n) * static_cast<double>(n);
    if (w <= 0) return nn;
    const int64_t kmax = (w - 1 < n - 1) ? w - 1 : n - 1;   // band diagonals 1..kmax each side
    // n + 2 * sum_{k=1..kmax} (n-k)
    const double band = static_cast<double>(n) +
                        2.0 * (static_cast<double>(kmax) * static_cast<double>(n) -
                               0.5 * static_cast<double>(kmax) * static_cast<double>(kmax + 1));
    return nn - band;
}

}  // namespace

void measures_from_hist(const uint64_t *diag, const uint64_t *vert, const uint64_t *white,
                        int64_t n, const rqa_params &p, rqa_measures *out) {
    const Moments d_all = moments(diag, n, 1);
    const Moments d_min = moments(diag, n, p.lmin);
    const Moments v_all = moments(vert, n, 1);
    const Moments v_min = moments(vert, n, p.vmin);
    const Moments w_min = moments(white, n, p.wmin);

    out->n_vec = n;
    out->n_rec = 0;
    for (int64_t l = 1; l <= n; ++l) out->n_rec += diag[l] * static_cast<uint64_t>(l);

    out->rr = ratio(d_all.mass, cells_outside_band(n, p.theiler));
    out->det = ratio(d_min.mass, d_all.mass);
    out->l = ratio(d_min.mass, d_min.count);
    out->lmax = longest(diag, n);
    out->div = out->lmax == 0.0 ? std::numeric_limits<double>::quiet_NaN() : 1.0 / out->lmax;
    out->l_entr = entropy(diag, n, p.lmin, d_min.count);
    out->lam = ratio(v_min.mass, v_all.mass);
    out->tt = ratio(v_min.mass, v_min.count);
    out->vmax = longest(vert, n);
    out->v_entr = entropy(vert, n, p.vmin, v_min.count);
    out->w = ratio(w_min.mass, w_min.count);
    out->wmax = longest(white, n);
    out->w_entr = entropy(white, n, p.wmin, w_min.count);
}

}  // namespace rqa
