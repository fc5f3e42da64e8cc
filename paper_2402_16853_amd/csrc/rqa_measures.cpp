// Host-side RQA measures in FP64 from the integer line-length histograms.
//
// Definitions: the measures listed in Tab. 3 (RR, DET, L, Lmax, DIV, L_entr,
// LAM, TT, Vmax, V_entr) plus the white-vertical analogues (W, Wmax, W_entr),
// derived from the frequency distributions of the three line types (Sect. 2).
// Sums run over ascending line length; empty denominators give NaN.
#include <algorithm>
#include <cmath>
#include <limits>

#include "rqa_internal.h"

namespace rqa {

namespace {

struct Moments {
    double count = 0.0;   // number of lines with length >= floor
    double mass = 0.0;    // sum of their lengths
};

// Shannon entropy (natural log) of the distribution of lines of length >= floor.
// A long histogram has ~10^5 classes, over which a running sum loses ~1e-11
// relative; the terms are summed as Ogita-Rump-Oishi "Sum2" (Knuth's
// error-free TwoSum per addition, the rounding errors accumulated apart and
// added at the end), which is as accurate as summing in twice the precision.
double entropy(const uint64_t *h, int64_t n, int64_t floor_len, double count) {
    if (count == 0.0) return std::numeric_limits<double>::quiet_NaN();
    double s = 0.0, err = 0.0;
    for (int64_t l = floor_len < 1 ? 1 : floor_len; l <= n; ++l) {
        if (h[l] == 0) continue;
        const double p = static_cast<double>(h[l]) / count;
        const double x = -(p * std::log(p));
        const double t = s + x;
        const double z = t - s;
        err += (s - (t - z)) + (x - z);
        s = t;
    }
    return s + err;
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

// Cells of an n_rows x n_cols matrix outside the band |i-j| < w: every cell
// minus the lengths of the band diagonals k = -(w-1) .. w-1.
double cells_outside_band_rect(int64_t n_rows, int64_t n_cols, int64_t w) {
    const double all = static_cast<double>(n_rows) * static_cast<double>(n_cols);
    if (w <= 0) return all;
    double band = 0.0;
    const int64_t klo = -std::min(w - 1, n_rows - 1), khi = std::min(w - 1, n_cols - 1);
    for (int64_t k = klo; k <= khi; ++k) {
        // diagonal k = j - i: rows max(0,-k) .. min(n_rows, n_cols - k) - 1
        const int64_t len = std::min(n_rows, n_cols - k) - std::max<int64_t>(0, -k);
        if (len > 0) band += static_cast<double>(len);
    }
    return all - band;
}

// Count, mass (sum of lengths), longest line and the count/mass over lengths
// >= floor, in one ascending pass.
struct Stats {
    Moments all;
    Moments min;
    double longest = 0.0;
};

Stats scan(const uint64_t *h, int64_t n, int64_t floor_len) {
    Stats st;
    for (int64_t l = 1; l <= n; ++l) {
        if (h[l] == 0) continue;
        const double c = static_cast<double>(h[l]);
        const double m = c * static_cast<double>(l);
        st.all.count += c;
        st.all.mass += m;
        if (l >= floor_len) {
            st.min.count += c;
            st.min.mass += m;
        }
        st.longest = static_cast<double>(l);
    }
    return st;
}

}  // namespace

void measures_from_hist(const uint64_t *diag, const uint64_t *vert, const uint64_t *white,
                        int64_t n, const rqa_params &p, rqa_measures *out) {
    const Stats d = scan(diag, n, p.lmin);
    const Stats v = scan(vert, n, p.vmin);
    const Stats w = scan(white, n, p.wmin);

    out->n_vec = n;
    out->n_rec = 0;
    for (int64_t l = 1; l <= n; ++l) out->n_rec += diag[l] * static_cast<uint64_t>(l);

    out->rr = ratio(d.all.mass, cells_outside_band(n, p.theiler));
    out->det = ratio(d.min.mass, d.all.mass);
    out->l = ratio(d.min.mass, d.min.count);
    out->lmax = d.longest;
    out->div = out->lmax == 0.0 ? std::numeric_limits<double>::quiet_NaN() : 1.0 / out->lmax;
    out->l_entr = entropy(diag, n, p.lmin, d.min.count);
    out->lam = ratio(v.min.mass, v.all.mass);
    out->tt = ratio(v.min.mass, v.min.count);
    out->vmax = v.longest;
    out->v_entr = entropy(vert, n, p.vmin, v.min.count);
    out->w = ratio(w.min.mass, w.min.count);
    out->wmax = w.longest;
    out->w_entr = entropy(white, n, p.wmin, w.min.count);
}

void measures_from_stats(const JobStats &st, int64_t n_rows, int64_t n_cols, const rqa_params &p,
                         rqa_measures *out) {
    const double nan = std::numeric_limits<double>::quiet_NaN();
    auto dbl = [](uint64_t v) { return static_cast<double>(v); };
    out->n_vec = n_rows;
    out->n_rec = st.mass_all[0];
    const double cells = n_rows == n_cols ? cells_outside_band(n_rows, p.theiler)
                                          : cells_outside_band_rect(n_rows, n_cols, p.theiler);
    out->rr = ratio(dbl(st.mass_all[0]), cells);
    out->det = ratio(dbl(st.mass_min[0]), dbl(st.mass_all[0]));
    out->l = ratio(dbl(st.mass_min[0]), dbl(st.cnt_min[0]));
    out->lmax = dbl(st.longest[0]);
    out->div = st.longest[0] == 0 ? nan : 1.0 / out->lmax;
    out->l_entr = st.cnt_min[0] ? st.ent[0] : nan;
    out->lam = ratio(dbl(st.mass_min[1]), dbl(st.mass_all[1]));
    out->tt = ratio(dbl(st.mass_min[1]), dbl(st.cnt_min[1]));
    out->vmax = dbl(st.longest[1]);
    out->v_entr = st.cnt_min[1] ? st.ent[1] : nan;
    out->w = ratio(dbl(st.mass_min[2]), dbl(st.cnt_min[2]));
    out->wmax = dbl(st.longest[2]);
    out->w_entr = st.cnt_min[2] ? st.ent[2] : nan;
}

}  // namespace rqa
