/*
 * dh_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU reference for the particle-pair
 * distance histogram. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it. The product library never links, loads or
 * calls it, and this file shares no code with it.
 *
 * What it computes (the definition, written out):
 *   * Histogram bins are half-open, [k*dr, (k+1)*dr) with dr = r_max/n_bins
 *     (Sec. 2.1, Eq. 4). Raw pair counts are returned, not the dr^-1
 *     normalised density, and r >= r_max is counted separately as
 *     out-of-range.
 *   * Pairs: for species s and t, all N_s*N_t pairs when s != t, and the
 *     N_s(N_s-1)/2 pairs with j > i when s == t (Sec. 2.2, Algorithm 1 and
 *     the single-species paragraph after it). One histogram per unordered
 *     species pair: (0,0),(1,1),...,(k-1,k-1) first, then (s,t) with s<t in
 *     lexicographic order.
 *   * Distance: difference vector from particle i to particle j, minimum
 *     image applied for periodic boxes, Euclidean length (Algorithm 1).
 *   * Minimum image (Sec. 2.3, Eq. 5): d' = d - B nint(B^-1 d), with B the
 *     matrix whose columns are the cell vectors a, b, c. For an orthorhombic
 *     cell B is diagonal. For a triclinic cell Eq. 5 is exact up to half the
 *     smallest cell width; beyond that the reduced vector is shifted to the
 *     26 neighbouring cells and the shortest image is kept (Sec. 2.3 last
 *     paragraph; Sec. 4.1 on the three-fold loop over neighbouring boxes).
 *     nint rounds half to even, as nearbyint() does in the default rounding
 *     mode (Sec. 4.1 names nearbyint()).
 *   * Bin index: kappa = (int)(n_bins * r / r_max) (Algorithm 1), evaluated
 *     as t = r * s with s = n_bins / r_max computed once; the pair is in range
 *     iff t < n_bins.
 *
 * Arithmetic: IEEE-754 binary64, round to nearest even, no contraction
 * (built with -ffp-contract=off), fma() only where written, sqrt() correctly
 * rounded. The exact op order is:
 *   d = x_j - x_i (per component)
 *   orthorhombic: n = nearbyint(d * (1/L)); d = fma(-L, n, d)
 *   triclinic:    sc = dz*h33; sb = fma(dz, h23, dy*h22);
 *                 sa = fma(dz, h13, fma(dy, h12, dx*h11)); n = nearbyint(s);
 *                 dz = fma(-cz, nc, dz); dy = fma(-cy, nc, fma(-by, nb, dy));
 *                 dx = fma(-cx, nc, fma(-bx, nb, fma(-ax, na, dx)))
 *   q = fma(dz, dz, fma(dy, dy, dx*dx)); image search: q = min over the
 *   shifts S = i*a + j*b + k*c (i, j, k in {-1,0,1}) of the same expression
 *   on d + S; r = sqrt(q); t = r * s.
 * with h = B^-1 for the upper-triangular B:
 *   h11 = 1/ax, h22 = 1/by, h33 = 1/cz, h12 = -bx/(ax*by),
 *   h23 = -cy/(by*cz), h13 = (bx*cy - by*cx)/(ax*by*cz).
 * The image search runs iff 2*r_max >= w_min*(1 - 1e-9), w_min being the
 * smallest face-to-face width of the cell.
 *
 * Edge pairs (for checking a reduced-precision histogram): a pair counts at
 * edge k (1 <= k <= n_bins) when |t - k| <= window * s.
 *
 * Parity pins: see tests/test_oracle_pins.py (exact rational brute force,
 * crafted integer distances, pair-count and species identities, box special
 * cases, the ideal-gas closed form, and planted mutants).
 *
 * Compile-time DHO_MUTANT=k plants a deliberate mistake (tests only).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef DHO_MUTANT
#define DHO_MUTANT 0
#endif

enum { DHO_BOX_NONE = 0, DHO_BOX_ORTHO = 1, DHO_BOX_TRICLINIC = 2 };
enum { DHO_IMAGES_PAPER = 0, DHO_IMAGES_27 = 1, DHO_IMAGES_125 = 2 };

typedef struct {
    int box_type;
    double ax, bx, by, cx, cy, cz;       /* cell rows a=(ax,0,0) b=(bx,by,0) c=(cx,cy,cz) */
    double L[3], iL[3];                  /* orthorhombic edges and reciprocals */
    double h11, h12, h13, h22, h23, h33; /* B^-1 */
    int n_shift;
    double shift[125][3];
    double s, nb;
} consts_t;

static int box_valid(int box_type, const double *box)
{
    if (box_type == DHO_BOX_NONE) return 1;
    if (!box) return 0;
    for (int k = 0; k < 9; ++k)
        if (!isfinite(box[k])) return 0;
    if (!(box[0] > 0 && box[4] > 0 && box[8] > 0)) return 0;
    if (box[1] != 0 || box[2] != 0 || box[5] != 0) return 0;
    if (box_type == DHO_BOX_ORTHO && (box[3] != 0 || box[6] != 0 || box[7] != 0)) return 0;
    return 1;
}

/* smallest face-to-face width of the cell spanned by rows a, b, c */
static double min_width(const double *box)
{
    const double *a = box, *b = box + 3, *c = box + 6;
    double bc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
    double ca[3] = {c[1] * a[2] - c[2] * a[1], c[2] * a[0] - c[0] * a[2], c[0] * a[1] - c[1] * a[0]};
    double ab[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    double vol = fabs(a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2]);
    double wa = vol / sqrt(bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
    double wb = vol / sqrt(ca[0] * ca[0] + ca[1] * ca[1] + ca[2] * ca[2]);
    double wc = vol / sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
    double w = wa < wb ? wa : wb;
    return w < wc ? w : wc;
}

static void make_consts(consts_t *k, int box_type, const double *box, double r_max,
                        int n_bins, int image_mode)
{
    memset(k, 0, sizeof(*k));
    k->box_type = box_type;
#if DHO_MUTANT == 11
    k->s = r_max / (double)n_bins;           /* mutant: inverted scale */
#else
    k->s = (double)n_bins / r_max;
#endif
    k->nb = (double)n_bins;
    if (box_type == DHO_BOX_NONE) return;
#if DHO_MUTANT == 3
    /* mutant: cell read as columns instead of rows (transposed) */
    k->ax = box[0]; k->bx = box[1]; k->by = box[4]; k->cx = box[2]; k->cy = box[5]; k->cz = box[8];
#else
    k->ax = box[0]; k->bx = box[3]; k->by = box[4]; k->cx = box[6]; k->cy = box[7]; k->cz = box[8];
#endif
    k->L[0] = k->ax; k->L[1] = k->by; k->L[2] = k->cz;
    for (int c = 0; c < 3; ++c) k->iL[c] = 1.0 / k->L[c];
    k->h11 = 1.0 / k->ax;
    k->h22 = 1.0 / k->by;
    k->h33 = 1.0 / k->cz;
    k->h12 = -k->bx / (k->ax * k->by);
    k->h23 = -k->cy / (k->by * k->cz);
    k->h13 = (k->bx * k->cy - k->by * k->cx) / (k->ax * k->by * k->cz);
#if DHO_MUTANT == 10
    k->h12 = 0.0; k->h13 = 0.0; k->h23 = 0.0;     /* mutant: diagonal inverse only */
#endif
    k->n_shift = 0;
    if (box_type == DHO_BOX_TRICLINIC) {
        int reach = 0;
        if (image_mode == DHO_IMAGES_27) reach = 1;
        else if (image_mode == DHO_IMAGES_125) reach = 2;
        else if (2.0 * r_max >= min_width(box) * (1.0 - 1e-9)) reach = 1;
#if DHO_MUTANT == 9
        reach = 0;                                 /* mutant: never search images */
#endif
        if (reach) {
            for (int i = -reach; i <= reach; ++i)
                for (int j = -reach; j <= reach; ++j)
                    for (int l = -reach; l <= reach; ++l) {
                        double *S = k->shift[k->n_shift++];
                        S[0] = (double)i * k->ax + (double)j * k->bx + (double)l * k->cx;
                        S[1] = (double)j * k->by + (double)l * k->cy;
                        S[2] = (double)l * k->cz;
                    }
        }
    }
}

static inline double nint(double v)
{
#if DHO_MUTANT == 7
    return trunc(v);                               /* mutant: truncation */
#else
    return nearbyint(v);
#endif
}

static inline double sq3(double x, double y, double z)
{
#if DHO_MUTANT == 1
    (void)z;
    return fma(y, y, x * x);                       /* mutant: dropped z term */
#else
    return fma(z, z, fma(y, y, x * x));
#endif
}

/* squared minimum-image distance from particle i to particle j */
static double pair_q(const consts_t *k, const double *xi, const double *xj)
{
    double dx = xj[0] - xi[0], dy = xj[1] - xi[1], dz = xj[2] - xi[2];
    if (k->box_type == DHO_BOX_ORTHO) {
        double n0 = nint(dx * k->iL[0]), n1 = nint(dy * k->iL[1]), n2 = nint(dz * k->iL[2]);
#if DHO_MUTANT == 2
        dx = fma(k->L[0], n0, dx); dy = fma(k->L[1], n1, dy); dz = fma(k->L[2], n2, dz);
#else
        dx = fma(-k->L[0], n0, dx); dy = fma(-k->L[1], n1, dy); dz = fma(-k->L[2], n2, dz);
#endif
    } else if (k->box_type == DHO_BOX_TRICLINIC) {
        double sc = dz * k->h33;
        double sb = fma(dz, k->h23, dy * k->h22);
        double sa = fma(dz, k->h13, fma(dy, k->h12, dx * k->h11));
        double na = nint(sa), nb = nint(sb), nc = nint(sc);
        dz = fma(-k->cz, nc, dz);
        dy = fma(-k->cy, nc, fma(-k->by, nb, dy));
        dx = fma(-k->cx, nc, fma(-k->bx, nb, fma(-k->ax, na, dx)));
    }
    double q = sq3(dx, dy, dz);
    for (int m = 0; m < k->n_shift; ++m) {
        const double *S = k->shift[m];
        double v = sq3(dx + S[0], dy + S[1], dz + S[2]);
        if (v < q) q = v;
    }
    return q;
}

static inline double pair_t(const consts_t *k, const double *xi, const double *xj)
{
    return sqrt(pair_q(k, xi, xj)) * k->s;
}

static inline int in_range(double t, double nb)
{
#if DHO_MUTANT == 6
    return t <= nb;                                /* mutant: closed upper edge */
#else
    return t < nb;
#endif
}

static inline int64_t bin_of(double t, int n_bins)
{
#if DHO_MUTANT == 5
    int64_t b = (int64_t)(t + 0.5);                /* mutant: rounding, not floor */
#else
    int64_t b = (int64_t)t;
#endif
#if DHO_MUTANT == 5 || DHO_MUTANT == 6
    if (b >= n_bins) b = n_bins - 1;
#else
    (void)n_bins;
#endif
    return b;
}

/* histogram order: intra (s,s) first, then (s,t) s<t lexicographically */
static void hist_species(int n_species, int h, int *s_out, int *t_out)
{
#if DHO_MUTANT == 8
    /* mutant: cross pairs first */
    int n_cross = n_species * (n_species - 1) / 2;
    if (h >= n_cross) { *s_out = *t_out = h - n_cross; return; }
    int idx = 0;
    for (int s = 0; s < n_species; ++s)
        for (int t = s + 1; t < n_species; ++t, ++idx)
            if (idx == h) { *s_out = s; *t_out = t; return; }
#else
    if (h < n_species) { *s_out = *t_out = h; return; }
    int idx = n_species;
    for (int s = 0; s < n_species; ++s)
        for (int t = s + 1; t < n_species; ++t, ++idx)
            if (idx == h) { *s_out = s; *t_out = t; return; }
#endif
}

static int check_args(const double *coords, const int64_t *offsets, int32_t n_species,
                      int32_t box_type, const double *box, double r_max, int32_t n_bins)
{
    if (!offsets || n_species < 1 || n_species > 64) return -1;
    if (offsets[0] != 0) return -1;
    for (int s = 0; s < n_species; ++s)
        if (offsets[s + 1] < offsets[s]) return -1;
    if (offsets[n_species] > 0 && !coords) return -1;
    if (!(r_max > 0) || !isfinite(r_max)) return -1;
    if (n_bins < 1) return -1;
    if (box_type < 0 || box_type > 2 || !box_valid(box_type, box)) return -1;
    return 0;
}

int dho_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * The histogram of every species pair.
 *   hist         [H][n_bins]   overwritten
 *   out_of_range [H]           overwritten (may be NULL)
 *   edges        [H][n_bins]   edge-pair counts, edge k at index k-1, when
 *                              edge_window > 0 (may be NULL)
 * Returns 0, or -1 on an invalid argument (outputs untouched).
 */
int dho_histogram(const double *coords, const int64_t *offsets, int32_t n_species,
                  int32_t box_type, const double *box, double r_max, int32_t n_bins,
                  int32_t image_mode, double edge_window,
                  uint64_t *hist, uint64_t *out_of_range, uint64_t *edges, int32_t n_threads)
{
    if (check_args(coords, offsets, n_species, box_type, box, r_max, n_bins) || !hist) return -1;
    consts_t k;
    make_consts(&k, box_type, box, r_max, n_bins, image_mode);
    const int n_hist = n_species * (n_species + 1) / 2;
    const int want_edges = edges != NULL && edge_window > 0;
    const double ws = edge_window * k.s;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#else
    n_threads = 1;
#endif
    memset(hist, 0, sizeof(uint64_t) * (size_t)n_hist * n_bins);
    if (out_of_range) memset(out_of_range, 0, sizeof(uint64_t) * n_hist);
    if (want_edges) memset(edges, 0, sizeof(uint64_t) * (size_t)n_hist * n_bins);

    for (int h = 0; h < n_hist; ++h) {
        int s = 0, t = 0;
        hist_species(n_species, h, &s, &t);
        const int64_t i_lo = offsets[s], i_hi = offsets[s + 1];
        const int64_t j_hi = offsets[t + 1];
        const int same = (s == t);
        uint64_t *H = hist + (size_t)h * n_bins;
        uint64_t *E = want_edges ? edges + (size_t)h * n_bins : NULL;
        uint64_t oor_total = 0;
#pragma omp parallel num_threads(n_threads) reduction(+ : oor_total)
        {
            uint64_t *ph = calloc((size_t)n_bins, sizeof(uint64_t));
            uint64_t *pe = want_edges ? calloc((size_t)n_bins, sizeof(uint64_t)) : NULL;
            uint64_t oor = 0;
#pragma omp for schedule(dynamic, 16)
            for (int64_t i = i_lo; i < i_hi; ++i) {
#if DHO_MUTANT == 4
                int64_t j0 = same ? i : offsets[t];        /* mutant: self pairs */
#else
                int64_t j0 = same ? i + 1 : offsets[t];
#endif
                const double *xi = coords + 3 * i;
                for (int64_t j = j0; j < j_hi; ++j) {
                    double tv = pair_t(&k, xi, coords + 3 * j);
                    if (in_range(tv, k.nb)) ph[bin_of(tv, n_bins)] += 1;
                    else oor += 1;
                    if (pe) {
                        double lo = ceil(tv - ws), hi = floor(tv + ws);
                        if (lo < 1) lo = 1;
                        if (hi > n_bins) hi = n_bins;
                        for (double e = lo; e <= hi; e += 1) pe[(int64_t)e - 1] += 1;
                    }
                }
            }
#pragma omp critical
            {
                for (int b = 0; b < n_bins; ++b) H[b] += ph[b];
                if (pe) for (int b = 0; b < n_bins; ++b) E[b] += pe[b];
            }
            oor_total += oor;
            free(ph);
            free(pe);
        }
        if (out_of_range) out_of_range[h] = oor_total;
    }
    return 0;
}

/*
 * Scaled distance t = r * n_bins / r_max for explicit index pairs (global
 * particle indices), for sampled checks of large frames.
 */
int dho_pair_t(const double *coords, int64_t n, int32_t box_type, const double *box,
               double r_max, int32_t n_bins, int32_t image_mode,
               const int64_t *pi, const int64_t *pj, int64_t n_pairs, double *t_out)
{
    int64_t off[2] = {0, n};
    if (check_args(coords, off, 1, box_type, box, r_max, n_bins) || !pi || !pj || !t_out) return -1;
    consts_t k;
    make_consts(&k, box_type, box, r_max, n_bins, image_mode);
    for (int64_t m = 0; m < n_pairs; ++m) {
        if (pi[m] < 0 || pi[m] >= n || pj[m] < 0 || pj[m] >= n) return -1;
        t_out[m] = pair_t(&k, coords + 3 * pi[m], coords + 3 * pj[m]);
    }
    return 0;
}

/* smallest face-to-face width (exported for tests of the image rule) */
double dho_min_width(const double *box) { return min_width(box); }

int dho_mutant(void) { return DHO_MUTANT; }
