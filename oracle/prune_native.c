/*
 * Occlusion statistics of one view in plain C, float64 (oracle; test
 * infrastructure only: nothing in the product path links or loads it).
 *
 * Section 4.3: every pixel blends the Gaussians assigned to it front to
 * back and stops once its accumulated opacity is close to one; a Gaussian
 * that no pixel of any view blends is pruned.  This is the same per-pixel
 * loop as oracle/render.py (readings R1-R5, R13 of the design notes), written
 * as the sequential loop the paper describes, one pixel at a time, for the
 * scene sizes where the vectorised torch oracle is too slow:
 *
 *   list   the visible surfels whose pixel rectangle contains the pixel, in
 *          ascending (float32 centre-depth bits, id) - the caller passes the
 *          visible surfels already in that order
 *   per entry, with x the pixel centre and d = ((x-cx)/fx, (y-cy)/fy, 1):
 *          (u, v, tau) solves [a_u a_v -d] (u, v, tau)^T = -p (Cramer's
 *          rule; a zero determinant gives G_s = 0), G_s = exp(-(u^2+v^2)/2),
 *          G_f = exp(-|x - c|^2), G = G_s if G_s >= G_f else G_f,
 *          a = min(alpha_max, o G); skipped when a < alpha_min; the pixel
 *          stops before the entry when T (1 - a) < t_min; otherwise
 *          hits += 1, max_alpha = max(., a), max_weight = max(., a T) and
 *          T *= 1 - a.
 *   ties   a reached entry within the relative windows tie_cut of alpha_min
 *          (o G) or tie_term of t_min (T (1 - a)) may be decided the other
 *          way in float32; then every later decision of the pixel may change
 *          too (a cutoff tie scales the transmittance of the later entries by
 *          1 - a), up to m more entries past the stop for m ties.  Each
 *          entry so exposed - from the pixel's first tie entry on, and the
 *          next m entries past the stop that pass the cutoff - adds one to
 *          its surfel's tie[], the most its hits can change by.
 *
 * Finding a pixel's list: the surfels are bucketed by the 8x8-pixel cells
 * their rectangles meet (a lookup aid only); a pixel scans its cell's
 * bucket, which keeps the caller's order, and keeps the entries whose
 * rectangle contains it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define CELL 8

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double* a, const double* b, double* out) {
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

/* n_vis visible surfels in list order: id[k] the surfel id, rect[4k..4k+3]
 * = (x_lo, x_hi, y_lo, y_hi) inclusive pixel rectangle, p/au/av [3k..] the
 * camera-space centre and tangent axes, ctr[2k..] the projected centre,
 * opac[k].  pix_mask[H*W] (NULL: every pixel) selects the pixels rendered.
 * The statistics arrays are indexed by surfel id and accumulated (+=, max).
 * Returns 0, or -1 when out of memory. */
int prune_view_stats(int64_t n_vis, const int64_t* id, const int32_t* rect, const double* p, const double* au,
                     const double* av, const double* ctr, const double* opac, double fx, double fy, double cx,
                     double cy, int32_t W, int32_t H, double alpha_min, double alpha_max, double t_min,
                     double tie_cut, double tie_term, const uint8_t* pix_mask, int64_t* hits, double* max_alpha,
                     double* max_weight, uint32_t* tie) {
    const int32_t cw = (W + CELL - 1) / CELL, ch = (H + CELL - 1) / CELL;
    const int64_t ncell = (int64_t)cw * ch;
    int64_t* start = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
    if (!start) return -1;
    /* bucket sizes, then the buckets in list order */
    for (int64_t k = 0; k < n_vis; ++k) {
        const int32_t* r = rect + 4 * k;
        for (int32_t y = r[2] / CELL; y <= r[3] / CELL; ++y)
            for (int32_t x = r[0] / CELL; x <= r[1] / CELL; ++x) start[(int64_t)y * cw + x + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
    int64_t* bucket = (int64_t*)malloc(sizeof(int64_t) * (size_t)(start[ncell] > 0 ? start[ncell] : 1));
    if (!fill || !bucket) {
        free(start);
        free(fill);
        free(bucket);
        return -1;
    }
    for (int64_t c = 0; c < ncell; ++c) fill[c] = start[c];
    for (int64_t k = 0; k < n_vis; ++k) {
        const int32_t* r = rect + 4 * k;
        for (int32_t y = r[2] / CELL; y <= r[3] / CELL; ++y)
            for (int32_t x = r[0] / CELL; x <= r[1] / CELL; ++x) bucket[fill[(int64_t)y * cw + x]++] = k;
    }
    for (int32_t j = 0; j < H; ++j) {
        for (int32_t i = 0; i < W; ++i) {
            if (pix_mask && !pix_mask[(int64_t)j * W + i]) continue;
            const double x = i + 0.5, y = j + 0.5;
            const double d[3] = {(x - cx) / fx, (y - cy) / fy, 1.0};
            const double md[3] = {-d[0], -d[1], -d[2]};
            const int64_t c = (int64_t)(j / CELL) * cw + i / CELL;
            double T = 1.0;
            int64_t ties = 0;        /* tie entries met so far at this pixel */
            int64_t past = -1;       /* entries still to mark past the stop (-1: not stopped) */
            for (int64_t b = start[c]; b < start[c + 1]; ++b) {
                const int64_t k = bucket[b];
                const int32_t* r = rect + 4 * k;
                if (i < r[0] || i > r[1] || j < r[2] || j > r[3]) continue;
                const double* pk = p + 3 * k;
                const double* uk = au + 3 * k;
                const double* vk = av + 3 * k;
                const double mp[3] = {-pk[0], -pk[1], -pk[2]};
                double c23[3], cb3[3];
                cross3(vk, md, c23);
                const double det = dot3(uk, c23);
                double Gs = 0.0;
                if (det != 0.0) {
                    cross3(mp, md, cb3);
                    const double u = dot3(mp, c23) / det;
                    const double v = dot3(uk, cb3) / det;
                    Gs = exp(-(u * u + v * v) / 2.0);
                }
                const double dx = x - ctr[2 * k], dy = y - ctr[2 * k + 1];
                const double Gf = exp(-(dx * dx + dy * dy));
                const double G = Gs >= Gf ? Gs : Gf;
                const double a_raw = opac[k] * G;
                const double a = a_raw < alpha_max ? a_raw : alpha_max;
                const int64_t g = id[k];
                if (past >= 0) {
                    /* past the stop: entries that pass the cutoff are exposed */
                    if (a >= alpha_min) {
                        tie[g] += 1;
                        if (--past == 0) break;
                    }
                    continue;
                }
                const int cut_tie = fabs(a_raw - alpha_min) <= tie_cut * alpha_min;
                if (a < alpha_min) {
                    /* a skip does not depend on the transmittance: only its own tie exposes it */
                    ties += cut_tie;
                    tie[g] += cut_tie;
                    continue;
                }
                const double Tn = T * (1.0 - a);
                ties += cut_tie || fabs(Tn - t_min) <= tie_term * t_min;
                tie[g] += ties > 0;
                if (Tn < t_min) {
                    if (ties == 0) break;
                    past = ties;
                    continue;
                }
                hits[g] += 1;
                if (a > max_alpha[g]) max_alpha[g] = a;
                if (a * T > max_weight[g]) max_weight[g] = a * T;
                T = Tn;
            }
        }
    }
    free(start);
    free(fill);
    free(bucket);
    return 0;
}
