/*
 * lse_oracle.c -- FP64 CPU oracle for the fast level set evolutions (LSE) of
 * Li, Shi, Wang and Miao, "Extracting Man-Made Objects From Remote Sensing
 * Images via Fast Level Set Evolutions" (arXiv 1409.7474).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may build, load or
 * call it; the product path never does.  It shares no code, header, table or
 * constant generator with the HIP library.
 *
 * Everything is double precision, written as the paper defines it:
 *   - the Gaussian template is the full ts x ts normalised 2-D template
 *     (Table I step 4 and Sec. III-D Step 4; the template-size parameter "TS"
 *     of Table III), applied as a DIRECT 2-D convolution with zero padding and
 *     same-size output (no separable shortcut);
 *   - gradients are first differences: central inside, one-sided at the image
 *     border (the gradient rule of the edge-LSE listing in the appendix);
 *   - region means follow eq. (15) (c+ on phi >= 0, c- on phi < 0, vector
 *     notation per band), the normalised region term follows eq. (17) with
 *     the sign of the algebraic expansion of eq. (15) (eq. (16) prints a "+"
 *     that the expansion does not give);
 *   - the edge term is g(I) of eq. (14);
 *   - one iteration follows Table I steps 2-4 (update, reinitialise to a
 *     binary function, Gaussian regularisation), the update being eq. (18).
 *
 * Readings where the paper is silent or self-contradictory (all listed in the
 * design notes): ties phi == 0 go to the + side everywhere; an empty region
 * has mean 0; M == 0 gives R == 0; the edge map is computed on the band mean
 * multiplied by an intensity scale (the listing works on 8-bit digital
 * numbers); a second step order (smooth, then binarise) reproduces the
 * appendix listing and is selected by order = 1.
 *
 * Reductions are done per row, then summed over rows in row order, so the
 * result does not depend on the number of OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(y, x, w) ((size_t)(y) * (size_t)(w) + (size_t)(x))

int lseo_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void lseo_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Normalised 2-D Gaussian template of side ts (odd), Sec. III-D Step 4 / Table
 * III "TS".  K[i*ts + j] = exp(-((i-r)^2 + (j-r)^2) / (2 sigma^2)) / sum. */
void lseo_template2d(double sigma, int ts, double *K) {
    int r = ts / 2;
    double s = 0.0;
    for (int i = 0; i < ts; ++i)
        for (int j = 0; j < ts; ++j) {
            double di = i - r, dj = j - r;
            double v = exp(-(di * di + dj * dj) / (2.0 * sigma * sigma));
            K[i * ts + j] = v;
            s += v;
        }
    for (int i = 0; i < ts * ts; ++i) K[i] /= s;
}

/* Direct 2-D convolution, same-size output, zero outside the image:
 * out(y,x) = sum_{i,j} K(i,j) f(y + r - i, x + r - j). */
void lseo_conv2_same(const double *f, int h, int w, const double *K, int ts, double *out) {
    int r = ts / 2;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < h; ++y) {
        for (int x = 0; x < w; ++x) {
            double acc = 0.0;
            for (int i = 0; i < ts; ++i) {
                int yy = y + r - i;
                if (yy < 0 || yy >= h) continue;
                for (int j = 0; j < ts; ++j) {
                    int xx = x + r - j;
                    if (xx < 0 || xx >= w) continue;
                    acc += K[i * ts + j] * f[IDX(yy, xx, w)];
                }
            }
            out[IDX(y, x, w)] = acc;
        }
    }
}

/* First differences: central inside, one-sided at the border.  fx runs along
 * a row (column index x), fy along a column (row index y).  h, w >= 2. */
void lseo_gradient(const double *f, int h, int w, double *fx, double *fy) {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < h; ++y) {
        for (int x = 0; x < w; ++x) {
            double gx, gy;
            if (x == 0)
                gx = f[IDX(y, 1, w)] - f[IDX(y, 0, w)];
            else if (x == w - 1)
                gx = f[IDX(y, w - 1, w)] - f[IDX(y, w - 2, w)];
            else
                gx = 0.5 * (f[IDX(y, x + 1, w)] - f[IDX(y, x - 1, w)]);
            if (y == 0)
                gy = f[IDX(1, x, w)] - f[IDX(0, x, w)];
            else if (y == h - 1)
                gy = f[IDX(h - 1, x, w)] - f[IDX(h - 2, x, w)];
            else
                gy = 0.5 * (f[IDX(y + 1, x, w)] - f[IDX(y - 1, x, w)]);
            fx[IDX(y, x, w)] = gx;
            fy[IDX(y, x, w)] = gy;
        }
    }
}

/* |grad f| with the rule above. */
void lseo_grad_mag(const double *f, int h, int w, double *mag) {
    size_t n = (size_t)h * w;
    double *fx = (double *)malloc(n * sizeof(double));
    double *fy = (double *)malloc(n * sizeof(double));
    lseo_gradient(f, h, w, fx, fy);
    for (size_t i = 0; i < n; ++i) mag[i] = sqrt(fx[i] * fx[i] + fy[i] * fy[i]);
    free(fx);
    free(fy);
}

/* Region means of eq. (15): c+_b = mean of I_b over {phi >= 0}, c-_b over
 * {phi < 0}; an empty region has mean 0.  I is h*w*nb, band fastest. */
void lseo_region_means(const double *I, int h, int w, int nb, const double *phi,
                       double *cplus, double *cminus, int64_t *nplus_out) {
    double *rs_p = (double *)calloc((size_t)h * nb, sizeof(double));
    double *rs_m = (double *)calloc((size_t)h * nb, sizeof(double));
    int64_t *rc = (int64_t *)calloc((size_t)h, sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int y = 0; y < h; ++y) {
        for (int x = 0; x < w; ++x) {
            const double *px = I + IDX(y, x, w) * nb;
            if (phi[IDX(y, x, w)] >= 0.0) {
                rc[y] += 1;
                for (int b = 0; b < nb; ++b) rs_p[(size_t)y * nb + b] += px[b];
            } else {
                for (int b = 0; b < nb; ++b) rs_m[(size_t)y * nb + b] += px[b];
            }
        }
    }
    int64_t np = 0;
    for (int y = 0; y < h; ++y) np += rc[y];
    int64_t nm = (int64_t)h * w - np;
    for (int b = 0; b < nb; ++b) {
        double sp = 0.0, sm = 0.0;
        for (int y = 0; y < h; ++y) {
            sp += rs_p[(size_t)y * nb + b];
            sm += rs_m[(size_t)y * nb + b];
        }
        cplus[b] = np > 0 ? sp / (double)np : 0.0;
        cminus[b] = nm > 0 ? sm / (double)nm : 0.0;
    }
    if (nplus_out) *nplus_out = np;
    free(rs_p);
    free(rs_m);
    free(rc);
}

/* Normalised region data term of eq. (17):
 *   D(x) = sum_b (c+_b - c-_b) (2 I_b(x) - c+_b - c-_b),
 *   M = max_x |D(x)|,  R = D / M  (R = 0 everywhere when M = 0). */
void lseo_region_term(const double *I, int h, int w, int nb, const double *cplus,
                      const double *cminus, double *R, double *M_out) {
    size_t n = (size_t)h * w;
    double M = 0.0;
    for (size_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int b = 0; b < nb; ++b)
            d += (cplus[b] - cminus[b]) * (2.0 * I[i * nb + b] - cplus[b] - cminus[b]);
        R[i] = d;
        if (fabs(d) > M) M = fabs(d);
    }
    for (size_t i = 0; i < n; ++i) R[i] = M > 0.0 ? R[i] / M : 0.0;
    if (M_out) *M_out = M;
}

/* Edge function g(I) of eq. (14), on the band-mean intensity times `scale`:
 *   Is = G_{sigma1} * (scale * mean_b I_b)   (direct 2-D, zero padding),
 *   g  = 1 / (1 + |grad Is|^2). */
void lseo_edge_map(const double *I, int h, int w, int nb, double sigma1, int ts1,
                   double scale, double *g) {
    size_t n = (size_t)h * w;
    double *gray = (double *)malloc(n * sizeof(double));
    double *Is = (double *)malloc(n * sizeof(double));
    double *fx = (double *)malloc(n * sizeof(double));
    double *fy = (double *)malloc(n * sizeof(double));
    double *K1 = (double *)malloc((size_t)ts1 * ts1 * sizeof(double));
    for (size_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += I[i * nb + b];
        gray[i] = scale * (s / nb);
    }
    lseo_template2d(sigma1, ts1, K1);
    lseo_conv2_same(gray, h, w, K1, ts1, Is);
    lseo_gradient(Is, h, w, fx, fy);
    for (size_t i = 0; i < n; ++i) g[i] = 1.0 / (1.0 + fx[i] * fx[i] + fy[i] * fy[i]);
    free(gray);
    free(Is);
    free(fx);
    free(fy);
    free(K1);
}

/* One iteration (Table I steps 2-4; update of eq. (18)).
 *
 *   term:   0 = region term of eq. (17), 1 = edge term of eq. (14) (g given).
 *   order:  0 = Table I (update, binarise, smooth);
 *           1 = appendix listing (update, smooth, binarise).
 *   reinit: 1 = binarise in this iteration, 0 = skip the binarisation
 *           (Sec. III-D Step 3 makes it optional for the region term).
 *
 * Inputs: phi (h*w), image I (h*w*nb, band fastest; region term), g (h*w;
 * edge term), K (ts*ts normalised template), dt.
 * Outputs (any may be NULL except phi_out):
 *   phi_out   the LSF after the iteration;
 *   u_out     phi + dt * R * |grad phi| (before binarisation/smoothing);
 *   psi_out   order 1 only: G * u, the field that is binarised;
 *   b_out     +1/-1 binary produced in this iteration (order 0: sign of u;
 *             order 1: sign of psi; no reinit: sign of phi_out);
 *   stats     [0..nb-1] c+, [4..4+nb-1] c-, [8] M, [9] N+ (region term;
 *             left untouched for the edge term).
 */
void lseo_step(const double *I, int h, int w, int nb, const double *g, int term, int order,
               int reinit, double dt, const double *K, int ts, const double *phi,
               double *phi_out, double *u_out, double *psi_out, int8_t *b_out, double *stats) {
    size_t n = (size_t)h * w;
    double *R = (double *)malloc(n * sizeof(double));
    double *mag = (double *)malloc(n * sizeof(double));
    double *u = (double *)malloc(n * sizeof(double));
    double *tmp = (double *)malloc(n * sizeof(double));

    /* Step 2.1: data term. */
    if (term == 0) {
        double cp[4] = {0, 0, 0, 0}, cm[4] = {0, 0, 0, 0}, M = 0.0;
        int64_t np = 0;
        lseo_region_means(I, h, w, nb, phi, cp, cm, &np);
        lseo_region_term(I, h, w, nb, cp, cm, R, &M);
        if (stats) {
            for (int b = 0; b < 4; ++b) {
                stats[b] = b < nb ? cp[b] : 0.0;
                stats[4 + b] = b < nb ? cm[b] : 0.0;
            }
            stats[8] = M;
            stats[9] = (double)np;
        }
    } else {
        memcpy(R, g, n * sizeof(double));
    }
    /* |grad phi| and step 2.2: explicit Euler update, eq. (18). */
    lseo_grad_mag(phi, h, w, mag);
    for (size_t i = 0; i < n; ++i) u[i] = phi[i] + dt * R[i] * mag[i];
    if (u_out) memcpy(u_out, u, n * sizeof(double));

    if (order == 0) {
        /* Step 3: reinitialise to a binary function (ties to +1). */
        if (reinit)
            for (size_t i = 0; i < n; ++i) tmp[i] = u[i] >= 0.0 ? 1.0 : -1.0;
        else
            memcpy(tmp, u, n * sizeof(double));
        /* Step 4: Gaussian regularisation. */
        lseo_conv2_same(tmp, h, w, K, ts, phi_out);
        if (b_out)
            for (size_t i = 0; i < n; ++i)
                b_out[i] = (int8_t)(reinit ? (tmp[i] > 0.0 ? 1 : -1) : (phi_out[i] >= 0.0 ? 1 : -1));
    } else {
        /* Listing order: smooth the updated LSF, then binarise it. */
        lseo_conv2_same(u, h, w, K, ts, tmp);
        if (psi_out) memcpy(psi_out, tmp, n * sizeof(double));
        for (size_t i = 0; i < n; ++i) phi_out[i] = reinit ? (tmp[i] >= 0.0 ? 1.0 : -1.0) : tmp[i];
        if (b_out)
            for (size_t i = 0; i < n; ++i) b_out[i] = (int8_t)(tmp[i] >= 0.0 ? 1 : -1);
    }
    free(R);
    free(mag);
    free(u);
    free(tmp);
}

/* Whole evolution (Table I steps 1-6).
 *   mask: h*w, nonzero = inside the initial curve (phi0 = +1, eq. (13)).
 *   reinit_every: 1 = binarise every iteration; k > 1 = every k-th iteration;
 *                 0 = never.
 *   stop_unchanged: stop after the first iteration whose binary result equals
 *                 the previous one (Step 5).
 * Outputs: phi_out (final LSF), b_out (+1/-1 binary result of the last
 * iteration; the initial mask if max_iters == 0), iters_done, and per
 * iteration flips (number of pixels whose binary result changed; may be NULL,
 * length max_iters). Returns 0. */
int lseo_run(const double *I, int h, int w, int nb, const double *g, int term, int order,
             int reinit_every, double dt, const double *K, int ts, const uint8_t *mask,
             int max_iters, int stop_unchanged, double *phi_out, int8_t *b_out,
             int *iters_done, int64_t *flips) {
    size_t n = (size_t)h * w;
    double *phi = (double *)malloc(n * sizeof(double));
    double *nxt = (double *)malloc(n * sizeof(double));
    int8_t *bprev = (int8_t *)malloc(n);
    int8_t *bcur = (int8_t *)malloc(n);
    for (size_t i = 0; i < n; ++i) {
        phi[i] = mask[i] ? 1.0 : -1.0; /* eq. (13) */
        bprev[i] = mask[i] ? 1 : -1;
    }
    int it = 0;
    for (; it < max_iters; ++it) {
        int reinit = reinit_every > 0 && ((it + 1) % reinit_every) == 0;
        lseo_step(I, h, w, nb, g, term, order, reinit, dt, K, ts, phi, nxt, NULL, NULL, bcur, NULL);
        int64_t fl = 0;
        for (size_t i = 0; i < n; ++i) fl += bcur[i] != bprev[i];
        if (flips) flips[it] = fl;
        double *t = phi;
        phi = nxt;
        nxt = t;
        int8_t *tb = bprev;
        bprev = bcur;
        bcur = tb;
        if (stop_unchanged && fl == 0) {
            ++it;
            break;
        }
    }
    memcpy(phi_out, phi, n * sizeof(double));
    if (b_out) memcpy(b_out, bprev, n);
    if (iters_done) *iters_done = it;
    free(phi);
    free(nxt);
    free(bprev);
    free(bcur);
    return 0;
}
