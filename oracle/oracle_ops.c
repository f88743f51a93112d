/*
 * FP64 CPU oracle: operators of the superiorized conjugate gradient method.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The product path (the
 * HIP library) never links, loads or calls it, and it shares no code, header,
 * table or constant generator with it.
 *
 * Plain loops in double precision, written for a reader to check by eye.
 * OpenMP only distributes independent rays / pixels / angles over threads; it
 * changes no arithmetic.
 *
 * Operators (paper, Introduction: the least-squares problem min 1/2||y-Ax||^2
 * with A an L x J system matrix that discretises the line integrals):
 *   or_project      y = A x     ray-driven: exact chords by Siddon traversal
 *   or_backproject  x = A^T y   pixel-driven: exact chords by slab clipping
 *   or_tv / or_tv_subgrad       isotropic total variation and a subgradient
 *   or_filter_kernel / or_filter  the preconditioning filter F^T C F applied
 *                               to each projection (Filters for
 *                               Preconditioning section, eq. of c(omega))
 *
 * Geometry (the paper fixes only parallel rays, angles uniform over
 * [0, 180 deg) and the image/detector sizes; the rest is this oracle's
 * reading):
 *   pixel (i, j) has centre x_j = j - (N-1)/2, y_i = (N-1)/2 - i and covers the
 *   closed unit square around it; angle a has theta_a = a*pi/n_a; bin b has
 *   centre t_b = b - (n_b-1)/2; ray (a, b) is the line
 *   {x cos theta_a + y sin theta_a = t_b}. A's entry for (ray, pixel) is the
 *   length of the ray inside the pixel square. A ray lying exactly on a pixel
 *   edge gives each of the two pixels half of the edge length.
 *   cos/sin are evaluated in double and snapped to 0 / +-1 within 1e-12, so
 *   the angles 0 and 90 degrees are exactly axis-aligned.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

static double snap(double v)
{
    if (fabs(v) < 1e-12) return 0.0;
    if (fabs(1.0 - fabs(v)) < 1e-12) return v > 0 ? 1.0 : -1.0;
    return v;
}

int or_trig(int n_angles, double *cosv, double *sinv)
{
    if (n_angles <= 0) return -1;
    for (int a = 0; a < n_angles; ++a) {
        double th = (double)a * OR_PI / (double)n_angles;
        cosv[a] = snap(cos(th));
        sinv[a] = snap(sin(th));
    }
    return 0;
}

static void set_threads(int threads)
{
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Ray-driven chords (Siddon): every crossing of the ray with a grid line is  */
/* found, the crossings are merged in order along the ray, and each piece     */
/* between consecutive crossings lies in one pixel, found from its midpoint.  */
/* ------------------------------------------------------------------------ */

/* Crossing parameters lambda of the line p(l) = p0 + l*d with the grid lines
 * coord = -B + k, k = 0..n, in increasing order of lambda. */
static int crossings(int n, double p0, double d, double B, double *out)
{
    int m = 0;
    if (d > 0) {
        for (int k = 0; k <= n; ++k) out[m++] = (-B + k - p0) / d;
    } else {
        for (int k = n; k >= 0; --k) out[m++] = (-B + k - p0) / d;
    }
    return m;
}

/* Emits (pixel, length) for ray (c, s, t). Buffers must hold 4n + 8 entries.
 * Returns the number of entries. */
static int siddon(int n, double c, double s, double t, double *lam_x, double *lam_y,
                  double *lam, int *pix, double *len)
{
    const double B = 0.5 * n;
    const double p0x = t * c, p0y = t * s;
    const double dx = -s, dy = c;
    double lo = -INFINITY, hi = INFINITY;

    /* Slab of the whole image along x. */
    if (dx != 0.0) {
        double l1 = (-B - p0x) / dx, l2 = (B - p0x) / dx;
        lo = fmax(lo, fmin(l1, l2));
        hi = fmin(hi, fmax(l1, l2));
    } else if (p0x < -B || p0x > B) {
        return 0;
    }
    if (dy != 0.0) {
        double l1 = (-B - p0y) / dy, l2 = (B - p0y) / dy;
        lo = fmax(lo, fmin(l1, l2));
        hi = fmin(hi, fmax(l1, l2));
    } else if (p0y < -B || p0y > B) {
        return 0;
    }
    if (!(hi > lo)) return 0;

    /* Merge the ordered crossings with x- and y-grid lines inside (lo, hi). */
    int mx = dx != 0.0 ? crossings(n, p0x, dx, B, lam_x) : 0;
    int my = dy != 0.0 ? crossings(n, p0y, dy, B, lam_y) : 0;
    int m = 0, ix = 0, iy = 0;
    lam[m++] = lo;
    while (ix < mx || iy < my) {
        double v;
        if (iy >= my || (ix < mx && lam_x[ix] <= lam_y[iy])) v = lam_x[ix++];
        else v = lam_y[iy++];
        if (v > lo && v < hi) lam[m++] = v;
    }
    lam[m++] = hi;

    int cnt = 0;
    for (int k = 0; k + 1 < m; ++k) {
        double l = lam[k + 1] - lam[k];
        if (!(l > 0.0)) continue;
        double lm = 0.5 * (lam[k] + lam[k + 1]);
        double px = p0x + lm * dx, py = p0y + lm * dy;
        /* Columns / rows touched by the piece. When the ray runs along a grid
         * line the piece lies on the edge of two pixels: half to each. */
        double u = px + B;           /* column coordinate, pixel j covers [j, j+1] */
        double w = B - py;           /* row coordinate,    pixel i covers [i, i+1] */
        int j0, j1, i0, i1;
        if (dx == 0.0 && u == floor(u)) { j0 = (int)u - 1; j1 = (int)u; }
        else { j0 = j1 = (int)floor(u); }
        if (dy == 0.0 && w == floor(w)) { i0 = (int)w - 1; i1 = (int)w; }
        else { i0 = i1 = (int)floor(w); }
        double share = 1.0;
        if (j0 != j1) share *= 0.5;
        if (i0 != i1) share *= 0.5;
        for (int ii = i0; ii <= i1; ++ii) {
            if (ii < 0 || ii >= n) continue;
            for (int jj = j0; jj <= j1; ++jj) {
                if (jj < 0 || jj >= n) continue;
                pix[cnt] = ii * n + jj;
                len[cnt] = share * l;
                ++cnt;
            }
        }
    }
    return cnt;
}

typedef struct {
    double *lam_x, *lam_y, *lam, *len;
    int *pix;
} siddon_buf;

static int buf_alloc(siddon_buf *b, int n)
{
    size_t m = (size_t)(4 * n + 8);
    b->lam_x = malloc(m * sizeof(double));
    b->lam_y = malloc(m * sizeof(double));
    b->lam = malloc(2 * m * sizeof(double));
    b->len = malloc(2 * m * sizeof(double));
    b->pix = malloc(2 * m * sizeof(int));
    return (b->lam_x && b->lam_y && b->lam && b->len && b->pix) ? 0 : -1;
}

static void buf_free(siddon_buf *b)
{
    free(b->lam_x); free(b->lam_y); free(b->lam); free(b->len); free(b->pix);
}

/* y[r] = sum over pixels of chord(r, pixel) * x[pixel] for the listed rays
 * (ray id r = a*n_bins + b). */
int or_project_rays(int n, int n_angles, int n_bins, const double *cosv, const double *sinv,
                    const double *x, const long long *rays, long long count, double *out,
                    int threads)
{
    int err = 0;
    (void)n_angles;
    set_threads(threads);
#pragma omp parallel reduction(| : err)
    {
        siddon_buf b;
        int ok = buf_alloc(&b, n) == 0;
        if (!ok) err = 1;
#pragma omp for schedule(dynamic, 64)
        for (long long q = 0; q < count; ++q) {
            if (!ok) continue;
            long long r = rays[q];
            int a = (int)(r / n_bins), bb = (int)(r % n_bins);
            double t = (double)bb - 0.5 * (n_bins - 1);
            int cnt = siddon(n, cosv[a], sinv[a], t, b.lam_x, b.lam_y, b.lam, b.pix, b.len);
            double acc = 0.0;
            for (int k = 0; k < cnt; ++k) acc += b.len[k] * x[b.pix[k]];
            out[q] = acc;
        }
        buf_free(&b);
    }
    return err ? -1 : 0;
}

int or_project(int n, int n_angles, int n_bins, const double *cosv, const double *sinv,
               const double *x, double *y, int threads)
{
    long long L = (long long)n_angles * n_bins;
    long long *rays = malloc((size_t)L * sizeof(long long));
    if (!rays) return -1;
    for (long long r = 0; r < L; ++r) rays[r] = r;
    int rc = or_project_rays(n, n_angles, n_bins, cosv, sinv, x, rays, L, y, threads);
    free(rays);
    return rc;
}

/* Dense A (L x J, row-major) from the Siddon chords; for tiny problems. */
int or_dense_matrix(int n, int n_angles, int n_bins, const double *cosv, const double *sinv,
                    double *A)
{
    long long J = (long long)n * n;
    siddon_buf b;
    if (buf_alloc(&b, n)) { buf_free(&b); return -1; }
    for (int a = 0; a < n_angles; ++a)
        for (int bb = 0; bb < n_bins; ++bb) {
            long long r = (long long)a * n_bins + bb;
            double *row = A + r * J;
            memset(row, 0, (size_t)J * sizeof(double));
            double t = (double)bb - 0.5 * (n_bins - 1);
            int cnt = siddon(n, cosv[a], sinv[a], t, b.lam_x, b.lam_y, b.lam, b.pix, b.len);
            for (int k = 0; k < cnt; ++k) row[b.pix[k]] += b.len[k];
        }
    buf_free(&b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Pixel-driven chords by clipping: for each pixel and angle, the line of     */
/* each nearby bin is clipped against the pixel square (slab method).         */
/* ------------------------------------------------------------------------ */

/* Interval of lambda for which p0 + lambda*d lies in the slab [lo, hi] of
 * one coordinate. *share becomes 1/2 when the line runs along an edge. */
static int slab(double p0, double d, double lo, double hi, double *l0, double *l1, double *share)
{
    if (d != 0.0) {
        double a = (lo - p0) / d, b = (hi - p0) / d;
        *l0 = fmin(a, b);
        *l1 = fmax(a, b);
        return 1;
    }
    *l0 = -INFINITY;
    *l1 = INFINITY;
    if (p0 > lo && p0 < hi) return 1;
    if (p0 == lo || p0 == hi) { *share *= 0.5; return 1; }
    return 0;
}

static double chord_in_square(double c, double s, double t, double xc, double yc)
{
    const double p0x = t * c, p0y = t * s, dx = -s, dy = c;
    double share = 1.0, ax, bx, ay, by;
    if (!slab(p0x, dx, xc - 0.5, xc + 0.5, &ax, &bx, &share)) return 0.0;
    if (!slab(p0y, dy, yc - 0.5, yc + 0.5, &ay, &by, &share)) return 0.0;
    double l = fmin(bx, by) - fmax(ax, ay);
    return l > 0.0 ? share * l : 0.0;
}

static double backproject_one(int n, int n_angles, int n_bins, const double *cosv,
                              const double *sinv, const double *y, long long p)
{
    const double h = 0.5 * (n - 1), hb = 0.5 * (n_bins - 1);
    int i = (int)(p / n), j = (int)(p % n);
    double xc = j - h, yc = h - i;
    double acc = 0.0;
    for (int a = 0; a < n_angles; ++a) {
        double c = cosv[a], s = sinv[a];
        double proj = xc * c + yc * s;       /* t of the line through the centre */
        /* The square's shadow on the detector is |t - proj| <= (|c|+|s|)/2;
         * bins just outside it are tested too (their chord is 0). */
        double reach = 0.5 * (fabs(c) + fabs(s)) + 1e-9;
        int b_lo = (int)ceil(proj + hb - reach), b_hi = (int)floor(proj + hb + reach);
        if (b_lo < 0) b_lo = 0;
        if (b_hi > n_bins - 1) b_hi = n_bins - 1;
        for (int b = b_lo; b <= b_hi; ++b) {
            double t = (double)b - hb;
            double w = chord_in_square(c, s, t, xc, yc);
            if (w != 0.0) acc += w * y[(long long)a * n_bins + b];
        }
    }
    return acc;
}

int or_backproject_pixels(int n, int n_angles, int n_bins, const double *cosv,
                          const double *sinv, const double *y, const long long *pixels,
                          long long count, double *out, int threads)
{
    set_threads(threads);
#pragma omp parallel for schedule(dynamic, 64)
    for (long long q = 0; q < count; ++q)
        out[q] = backproject_one(n, n_angles, n_bins, cosv, sinv, y, pixels[q]);
    return 0;
}

int or_backproject(int n, int n_angles, int n_bins, const double *cosv, const double *sinv,
                   const double *y, double *x, int threads)
{
    long long J = (long long)n * n;
    set_threads(threads);
#pragma omp parallel for schedule(dynamic, 64)
    for (long long p = 0; p < J; ++p)
        x[p] = backproject_one(n, n_angles, n_bins, cosv, sinv, y, p);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Total variation (the secondary criterion; the paper names it but does not  */
/* define its discretisation). Reading: isotropic forward differences over    */
/* the (N-1)^2 interior terms,                                                */
/*   TV(x) = sum_{i,j < N-1} sqrt(a_ij^2 + b_ij^2 + kappa^2),                 */
/*   a_ij = x[i+1][j] - x[i][j],  b_ij = x[i][j+1] - x[i][j].                 */
/* kappa = 0 gives the exact TV; kappa > 0 is the smoothing of the paper's    */
/* eq. for the NLCG weights.                                                  */
/* ------------------------------------------------------------------------ */

double or_tv(int n, const double *x, double kappa)
{
    double acc = 0.0;
    for (int i = 0; i + 1 < n; ++i)
        for (int j = 0; j + 1 < n; ++j) {
            double a = x[(i + 1) * n + j] - x[i * n + j];
            double b = x[i * n + j + 1] - x[i * n + j];
            acc += sqrt(a * a + b * b + kappa * kappa);
        }
    return acc;
}

/* A subgradient of TV: for each term t_ij, d t_ij / d x is -(a+b)/t at
 * (i, j), a/t at (i+1, j) and b/t at (i, j+1). A term with t = 0 contributes
 * 0, which lies in its subdifferential. */
void or_tv_subgrad(int n, const double *x, double kappa, double *s)
{
    memset(s, 0, (size_t)n * n * sizeof(double));
    for (int i = 0; i + 1 < n; ++i)
        for (int j = 0; j + 1 < n; ++j) {
            double a = x[(i + 1) * n + j] - x[i * n + j];
            double b = x[i * n + j + 1] - x[i * n + j];
            double t = sqrt(a * a + b * b + kappa * kappa);
            if (t == 0.0) continue;
            s[i * n + j] -= (a + b) / t;
            s[(i + 1) * n + j] += a / t;
            s[i * n + j + 1] += b / t;
        }
}

/* ------------------------------------------------------------------------ */
/* Preconditioning filter (Filters for Preconditioning section): per          */
/* projection, F is the DFT of the projection zero-padded to P samples, C is  */
/* the diagonal of c(w) = (|w| + mu)(0.54 + 0.46 cos w) at w_m = 2 pi m / P,  */
/* m = -P/2 .. P/2-1, and F^T is the inverse DFT followed by keeping the      */
/* first n_bins samples. Since P >= 2 n_bins - 1 this equals the linear       */
/* convolution with k[d] = (1/P) sum_m c(w_m) cos(w_m d), |d| < n_bins.        */
/* ------------------------------------------------------------------------ */

void or_filter_kernel(int n_bins, int P, double mu, double *k)
{
    for (int d = 0; d < n_bins; ++d) {
        double acc = 0.0;
        for (int m = -P / 2; m < P / 2; ++m) {
            double w = 2.0 * OR_PI * (double)m / (double)P;
            double cw = (fabs(w) + mu) * (0.54 + 0.46 * cos(w));
            acc += cw * cos(w * (double)d);
        }
        k[d] = acc / (double)P;
    }
}

int or_filter(int n_angles, int n_bins, const double *k, const double *r, double *out,
              int threads)
{
    set_threads(threads);
#pragma omp parallel for schedule(static)
    for (int a = 0; a < n_angles; ++a) {
        const double *ra = r + (long long)a * n_bins;
        double *oa = out + (long long)a * n_bins;
        for (int b = 0; b < n_bins; ++b) {
            double acc = 0.0;
            for (int bp = 0; bp < n_bins; ++bp) acc += k[abs(b - bp)] * ra[bp];
            oa[b] = acc;
        }
    }
    return 0;
}
