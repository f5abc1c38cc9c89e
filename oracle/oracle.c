/*
 * FP64 CPU oracle for the induced-dipole solve of a Thole-damped point-dipole
 * (AMOEBA-type) polarizable force field under Ewald summation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it exists so that tests and the benchmark's CPU-baseline leg
 * can check the GPU path against a slow, plainly written definition.  It shares
 * no code, header or table with the HIP sources.
 *
 * What it follows (the paper prints no formula of the polarization model; it
 * points to the standard works, whose published forms are written out here):
 *  - the split of electrostatics into real-space pairs and a reciprocal part
 *    (paper, "Global scheme" and "Real space scheme");
 *  - real-space screened radial functions B0..B3 of the Ewald sum, obtained by
 *    repeated differentiation of erfc(beta r)/r;
 *  - Thole damping of Ren & Ponder (2003) for AMOEBA: smeared charge density
 *    proportional to exp(-a u^3), u = r / (alpha_i alpha_j)^(1/6), giving the
 *    factors lambda3, lambda5, lambda7 on the 1/r^3, 3/r^5, 15/r^7 tensors;
 *  - the reciprocal part as a direct Ewald k-sum with tin-foil boundary (exact
 *    up to the k truncation), and the Gaussian self field of a dipole;
 *  - smooth PME of Essmann et al. (1995), paper "Reciprocal space scheme":
 *    cardinal B-splines of order n spread the multipolar density onto a grid,
 *    the potential on the grid comes from an FFT convolution (done by the
 *    Python side with numpy's FFT), and the field is gathered back with the
 *    spline derivatives;
 *  - the scaled-pair correction applied in a separate pass (paper, final real
 *    space scheme listing and its "correct_scaling" step).
 *
 * Units: Angstrom, e, e*A, e*A^2, A^3; fields in e/A^2.  Quadrupoles are the
 * traceless Theta with point potential Theta:rr / r^5, stored xx,xy,xz,yy,yz,zz.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* Minimum-image displacement; box == NULL means free space (no images). */
static void min_image(double d[3], const double *box)
{
    if (!box)
        return;
    for (int a = 0; a < 3; ++a)
        d[a] -= box[a] * round(d[a] / box[a]);
}

/* Thole damping of the 1/r^3, 3/r^5 and 15/r^7 tensors.  Returns 1 - lambda_k
 * (the screened-out fraction) to avoid cancellation:  eps = a u^3,
 * 1-l3 = e^-eps, 1-l5 = (1+eps) e^-eps, 1-l7 = (1+eps+3/5 eps^2) e^-eps.
 * Pair rule: a = min(a_i, a_j).  alpha_i alpha_j = 0 means no damping. */
void orc_thole_oml(double r, double alpha_i, double alpha_j, double a_i, double a_j, double oml[3])
{
    double damp = pow(alpha_i * alpha_j, 1.0 / 6.0);
    if (damp == 0.0) {
        oml[0] = oml[1] = oml[2] = 0.0;
        return;
    }
    double a = a_i < a_j ? a_i : a_j;
    double u = r / damp;
    double eps = a * u * u * u;
    double e = exp(-eps);
    oml[0] = e;
    oml[1] = (1.0 + eps) * e;
    oml[2] = (1.0 + eps + 0.6 * eps * eps) * e;
}

/* Ewald real-space radial functions: B0 = erfc(beta r)/r and
 * B_n = ((2n-1) B_{n-1} + (2 beta^2)^n exp(-beta^2 r^2)/(beta sqrt(pi))) / r^2.
 * With beta = 0 these are the bare 1/r, 1/r^3, 3/r^5, 15/r^7. */
static void ewald_b(double r, double beta, double b[4])
{
    double r2 = r * r;
    double g = beta > 0.0 ? 2.0 * beta / sqrt(ORC_PI) * exp(-beta * beta * r2) : 0.0;
    double t = 2.0 * beta * beta;
    b[0] = erfc(beta * r) / r;
    b[1] = (b[0] + g) / r2;
    b[2] = (3.0 * b[1] + t * g) / r2;
    b[3] = (5.0 * b[2] + t * t * g) / r2;
}

void orc_ewald_b(double r, double beta, double b[4]) { ewald_b(r, beta, b); }

/* Scale of pair (i,j) for the permanent field from the CSR of scaled pairs (1 if absent). */
static double pair_scale(int i, int j, const int32_t *ptr, const int32_t *sj, const double *ss)
{
    if (!ptr)
        return 1.0;
    for (int k = ptr[i]; k < ptr[i + 1]; ++k)
        if (sj[k] == j)
            return ss[k];
    return 1.0;
}

/*
 * Partner search of the real-space loops.  Without cells (nc == NULL) every other atom is a
 * candidate: the plain O(N^2) definition.  With cells, the atoms are binned (by the caller) in a
 * periodic grid of nc[0] x nc[1] x nc[2] cells, every cell at least rc wide and at least three
 * per axis; an atom in cell (cx, cy, cz) then finds every partner closer than rc under the
 * minimum image in the 27 cells (cx + {-1,0,1}, ...) taken modulo nc, each of them visited once.
 * The candidates are written to buf (room for n - 1) and their count returned.  Both searches
 * give the same pairs; only the order of the sums differs.
 */
static int partners(int i, int n, const int32_t *nc, const int32_t *cell_of, const int32_t *cell_start,
                    const int32_t *cell_atoms, int32_t *buf)
{
    int m = 0;
    if (!nc) {
        for (int j = 0; j < n; ++j)
            if (j != i)
                buf[m++] = j;
        return m;
    }
    int c = cell_of[i];
    int cz = c % nc[2], cy = (c / nc[2]) % nc[1], cx = c / (nc[1] * nc[2]);
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
            for (int e = -1; e <= 1; ++e) {
                int x = (cx + a + nc[0]) % nc[0], y = (cy + b + nc[1]) % nc[1], z = (cz + e + nc[2]) % nc[2];
                int cell = (x * nc[1] + y) * nc[2] + z;
                for (int k = cell_start[cell]; k < cell_start[cell + 1]; ++k)
                    if (cell_atoms[k] != i)
                        buf[m++] = cell_atoms[k];
            }
    return m;
}

/*
 * Real-space field of induced dipoles mu at the requested atoms:
 *   E_i = sum_{j != i, |r| < rc} ( -B1' mu_j + B2' (mu_j . r) r ),  r = r_i - r_j (minimum image),
 *   B1' = B1 - (1-l3)/r^3,  B2' = B2 - 3 (1-l5)/r^5.
 * Every pair is Thole-damped and unscaled.  out_idx == NULL: all atoms in order.
 */
void orc_real_mutual(int n, const double *pos, const double *box, double beta, double rc,
                     const double *alpha, const double *thole, const double *mu,
                     int n_out, const int32_t *out_idx, double *out,
                     const int32_t *nc, const int32_t *cell_of, const int32_t *cell_start,
                     const int32_t *cell_atoms)
{
#pragma omp parallel
    {
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 1 ? n : 1));
#pragma omp for schedule(dynamic, 8)
    for (int o = 0; o < n_out; ++o) {
        int i = out_idx ? out_idx[o] : o;
        double e[3] = {0.0, 0.0, 0.0};
        int m = partners(i, n, nc, cell_of, cell_start, cell_atoms, cand);
        for (int c = 0; c < m; ++c) {
            int j = cand[c];
            double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                           pos[3 * i + 2] - pos[3 * j + 2]};
            min_image(d, box);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double r = sqrt(r2);
            if (!(r < rc))
                continue;
            double b[4], oml[3];
            ewald_b(r, beta, b);
            orc_thole_oml(r, alpha[i], alpha[j], thole[i], thole[j], oml);
            double r3 = r2 * r, r5 = r3 * r2;
            double b1 = b[1] - oml[0] / r3;
            double b2 = b[2] - 3.0 * oml[1] / r5;
            const double *m = mu + 3 * j;
            double mr = m[0] * d[0] + m[1] * d[1] + m[2] * d[2];
            for (int a = 0; a < 3; ++a)
                e[a] += -b1 * m[a] + b2 * mr * d[a];
        }
        out[3 * o] = e[0];
        out[3 * o + 1] = e[1];
        out[3 * o + 2] = e[2];
    }
    free(cand);
    }
}

/*
 * Real-space permanent field (charge q, dipole d, traceless quadrupole Theta) at the
 * requested atoms, including the scaled-pair correction:
 *   E_i += q_j B1' r - B1' d_j + B2' (d_j.r) r + (1/3) B3' (Theta_j:rr) r - (2/3) B2' Theta_j r
 * with  Bn' = [r < rc] Bn - c_n (1 - s lambda_{2n+1}) / r^{2n+1},  c = 1, 3, 15,
 * s = the pair's scale (1 unless listed).  A listed pair is corrected even beyond rc,
 * so the reciprocal part's share of it is always removed: the pairs within rc come from the
 * partner search, the listed pairs at or beyond rc from the atom's row of the CSR.
 */
static void perm_pair(const double d[3], double r, int in_cut, double s, double beta, int i, int j,
                      const double *alpha, const double *thole, const double *q, const double *dip,
                      const double *quad, double e[3])
{
    double b[4] = {0.0, 0.0, 0.0, 0.0}, oml[3];
    if (in_cut)
        ewald_b(r, beta, b);
    orc_thole_oml(r, alpha[i], alpha[j], thole[i], thole[j], oml);
    double r2 = r * r, r3 = r2 * r, r5 = r3 * r2, r7 = r5 * r2;
    double b1 = b[1] - (1.0 - s * (1.0 - oml[0])) / r3;
    double b2 = b[2] - 3.0 * (1.0 - s * (1.0 - oml[1])) / r5;
    double b3 = b[3] - 15.0 * (1.0 - s * (1.0 - oml[2])) / r7;
    double qj = q ? q[j] : 0.0;
    double dj[3] = {0.0, 0.0, 0.0};
    if (dip)
        for (int a = 0; a < 3; ++a)
            dj[a] = dip[3 * j + a];
    double th[3][3] = {{0}};
    if (quad) {
        const double *t = quad + 6 * j;
        th[0][0] = t[0]; th[0][1] = th[1][0] = t[1]; th[0][2] = th[2][0] = t[2];
        th[1][1] = t[3]; th[1][2] = th[2][1] = t[4]; th[2][2] = t[5];
    }
    double dr = dj[0] * d[0] + dj[1] * d[1] + dj[2] * d[2];
    double thr[3], thrr = 0.0;
    for (int a = 0; a < 3; ++a) {
        thr[a] = th[a][0] * d[0] + th[a][1] * d[1] + th[a][2] * d[2];
        thrr += thr[a] * d[a];
    }
    for (int a = 0; a < 3; ++a)
        e[a] += qj * b1 * d[a] - b1 * dj[a] + b2 * dr * d[a] + b3 * thrr * d[a] / 3.0
                - 2.0 * b2 * thr[a] / 3.0;
}

void orc_real_perm(int n, const double *pos, const double *box, double beta, double rc,
                   const double *alpha, const double *thole, const double *q, const double *dip,
                   const double *quad, const int32_t *sc_ptr, const int32_t *sc_j, const double *sc_s,
                   int n_out, const int32_t *out_idx, double *out,
                   const int32_t *nc, const int32_t *cell_of, const int32_t *cell_start,
                   const int32_t *cell_atoms)
{
#pragma omp parallel
    {
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 1 ? n : 1));
#pragma omp for schedule(dynamic, 8)
    for (int o = 0; o < n_out; ++o) {
        int i = out_idx ? out_idx[o] : o;
        double e[3] = {0.0, 0.0, 0.0};
        int m = partners(i, n, nc, cell_of, cell_start, cell_atoms, cand);
        for (int c = 0; c < m; ++c) {
            int j = cand[c];
            double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                           pos[3 * i + 2] - pos[3 * j + 2]};
            min_image(d, box);
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (!(r < rc))
                continue;
            perm_pair(d, r, 1, pair_scale(i, j, sc_ptr, sc_j, sc_s), beta, i, j, alpha, thole, q, dip, quad, e);
        }
        if (sc_ptr)
            for (int k = sc_ptr[i]; k < sc_ptr[i + 1]; ++k) {
                int j = sc_j[k];
                double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                               pos[3 * i + 2] - pos[3 * j + 2]};
                min_image(d, box);
                double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                if (r < rc || sc_s[k] == 1.0)
                    continue;
                perm_pair(d, r, 0, sc_s[k], beta, i, j, alpha, thole, q, dip, quad, e);
            }
        out[3 * o] = e[0];
        out[3 * o + 1] = e[1];
        out[3 * o + 2] = e[2];
    }
    free(cand);
    }
}

/*
 * Reciprocal-space field by the direct Ewald sum over k = 2 pi (n1/Lx, n2/Ly, n3/Lz), 0 < |k| <= kmax,
 * tin-foil boundary, k = 0 omitted:
 *   E(r_i) = (4 pi / V) sum_k exp(-k^2 / 4 beta^2) / k^2 * k * Im[ rho(k) exp(i k.r_i) ],
 *   rho(k) = sum_j ( q_j - i k.d_j - (1/3) k.Theta_j.k ) exp(-i k.r_j).
 * The sum runs over one half-space of k and doubles it (rho(-k) = conj rho(k)).
 * q, dip, quad may be NULL (absent).  This does not include the self field.
 */
void orc_ksum_field(int n, const double *pos, const double *box, double beta, double kmax,
                    const double *q, const double *dip, const double *quad,
                    int n_out, const int32_t *out_idx, double *out)
{
    double vol = box[0] * box[1] * box[2];
    double kb[3] = {2.0 * ORC_PI / box[0], 2.0 * ORC_PI / box[1], 2.0 * ORC_PI / box[2]};
    int nm[3];
    for (int a = 0; a < 3; ++a)
        nm[a] = (int)ceil(kmax / kb[a]);
    for (int o = 0; o < 3 * n_out; ++o)
        out[o] = 0.0;
    int n1span = nm[0] + 1;
#pragma omp parallel
    {
        double *acc = (double *)calloc((size_t)3 * n_out, sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int i1 = 0; i1 < n1span; ++i1) {
            for (int i2 = -nm[1]; i2 <= nm[1]; ++i2) {
                for (int i3 = -nm[2]; i3 <= nm[2]; ++i3) {
                    /* half space: (i1 > 0) or (i1 == 0, i2 > 0) or (i1 == 0, i2 == 0, i3 > 0) */
                    if (i1 == 0 && (i2 < 0 || (i2 == 0 && i3 <= 0)))
                        continue;
                    double k[3] = {i1 * kb[0], i2 * kb[1], i3 * kb[2]};
                    double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                    if (k2 > kmax * kmax)
                        continue;
                    double f = 2.0 * (4.0 * ORC_PI / vol) * exp(-k2 / (4.0 * beta * beta)) / k2;
                    double sre = 0.0, sim = 0.0;
                    for (int j = 0; j < n; ++j) {
                        double th = k[0] * pos[3 * j] + k[1] * pos[3 * j + 1] + k[2] * pos[3 * j + 2];
                        double A = q ? q[j] : 0.0, B = 0.0;
                        if (quad) {
                            const double *t = quad + 6 * j;
                            double kqk = t[0] * k[0] * k[0] + t[3] * k[1] * k[1] + t[5] * k[2] * k[2]
                                         + 2.0 * (t[1] * k[0] * k[1] + t[2] * k[0] * k[2] + t[4] * k[1] * k[2]);
                            A -= kqk / 3.0;
                        }
                        if (dip)
                            B = -(k[0] * dip[3 * j] + k[1] * dip[3 * j + 1] + k[2] * dip[3 * j + 2]);
                        double c = cos(th), s = sin(th);
                        /* (A + iB)(c - i s) */
                        sre += A * c + B * s;
                        sim += B * c - A * s;
                    }
                    for (int o = 0; o < n_out; ++o) {
                        int i = out_idx ? out_idx[o] : o;
                        double ph = k[0] * pos[3 * i] + k[1] * pos[3 * i + 1] + k[2] * pos[3 * i + 2];
                        double im = sre * sin(ph) + sim * cos(ph);
                        for (int a = 0; a < 3; ++a)
                            acc[3 * o + a] += f * k[a] * im;
                    }
                }
            }
        }
#pragma omp critical
        for (int o = 0; o < 3 * n_out; ++o)
            out[o] += acc[o];
        free(acc);
    }
}

/* Cardinal B-spline M_n(x) by the recursion M_n(x) = [x M_{n-1}(x) + (n-x) M_{n-1}(x-1)] / (n-1),
 * with M_2 the hat function on [0, 2].  Derivatives: M_n' = M_{n-1}(x) - M_{n-1}(x-1),
 * M_n'' = M_{n-2}(x) - 2 M_{n-2}(x-1) + M_{n-2}(x-2).  (Essmann et al. 1995.) */
static double bspline(int n, double x)
{
    if (n == 2)
        return (x > 0.0 && x < 2.0) ? 1.0 - fabs(x - 1.0) : 0.0;
    return (x * bspline(n - 1, x) + (n - x) * bspline(n - 1, x - 1.0)) / (n - 1);
}

double orc_bspline(int n, double x, int deriv)
{
    if (deriv == 0)
        return bspline(n, x);
    if (deriv == 1)
        return bspline(n - 1, x) - bspline(n - 1, x - 1.0);
    if (deriv == 2)
        return bspline(n - 2, x) - 2.0 * bspline(n - 2, x - 1.0) + bspline(n - 2, x - 2.0);
    return bspline(n - 3, x) - 3.0 * bspline(n - 3, x - 1.0) + 3.0 * bspline(n - 3, x - 2.0) - bspline(n - 3, x - 3.0);
}

/* For one coordinate: scaled fractional u = K x / L wrapped into [0, K); the n grid lines that
 * carry weight are k_t = floor(u) - t (mod K), t = 0..n-1, with argument x_t = u - floor(u) + t. */
static void spline_axis(double x, double len, int kdim, int order, int *kidx, double *m0, double *m1,
                        double *m2)
{
    double u = kdim * (x / len);
    u -= kdim * floor(u / kdim);
    double fl = floor(u);
    double fr = u - fl;
    for (int t = 0; t < order; ++t) {
        int k = (int)fl - t;
        k = ((k % kdim) + kdim) % kdim;
        kidx[t] = k;
        double arg = fr + t;
        m0[t] = orc_bspline(order, arg, 0);
        m1[t] = orc_bspline(order, arg, 1) * kdim / len;
        m2[t] = orc_bspline(order, arg, 2) * (kdim / len) * (kdim / len);
    }
}

/*
 * Smooth-PME spread of the multipolar density onto a real grid Q[K0][K1][K2] (C order):
 *   Q(k) = sum_j [ q_j + d_j . grad_j + (1/3) Theta_j : grad_j grad_j ] W(k; r_j),
 *   W(k; r) = prod_a M_n(u_a(r) - k_a) over periodic images of k.
 * Q is zeroed first.  q, dip, quad may be NULL.  Serial (atomicity is not a concern here).
 */
void orc_spme_spread(int n, const double *pos, const double *box, const int32_t *kdim, int order,
                     const double *q, const double *dip, const double *quad, double *grid)
{
    size_t npts = (size_t)kdim[0] * kdim[1] * kdim[2];
    memset(grid, 0, npts * sizeof(double));
    int kx[8], ky[8], kz[8];
    double m0[3][8], m1[3][8], m2[3][8];
    for (int j = 0; j < n; ++j) {
        spline_axis(pos[3 * j], box[0], kdim[0], order, kx, m0[0], m1[0], m2[0]);
        spline_axis(pos[3 * j + 1], box[1], kdim[1], order, ky, m0[1], m1[1], m2[1]);
        spline_axis(pos[3 * j + 2], box[2], kdim[2], order, kz, m0[2], m1[2], m2[2]);
        double qj = q ? q[j] : 0.0;
        double dj[3] = {0.0, 0.0, 0.0};
        if (dip)
            for (int a = 0; a < 3; ++a)
                dj[a] = dip[3 * j + a];
        double t[6] = {0, 0, 0, 0, 0, 0};
        if (quad)
            for (int a = 0; a < 6; ++a)
                t[a] = quad[6 * j + a];
        for (int a = 0; a < order; ++a)
            for (int b = 0; b < order; ++b)
                for (int c = 0; c < order; ++c) {
                    double w = m0[0][a] * m0[1][b] * m0[2][c];
                    double wx = m1[0][a] * m0[1][b] * m0[2][c];
                    double wy = m0[0][a] * m1[1][b] * m0[2][c];
                    double wz = m0[0][a] * m0[1][b] * m1[2][c];
                    double wxx = m2[0][a] * m0[1][b] * m0[2][c];
                    double wyy = m0[0][a] * m2[1][b] * m0[2][c];
                    double wzz = m0[0][a] * m0[1][b] * m2[2][c];
                    double wxy = m1[0][a] * m1[1][b] * m0[2][c];
                    double wxz = m1[0][a] * m0[1][b] * m1[2][c];
                    double wyz = m0[0][a] * m1[1][b] * m1[2][c];
                    double v = qj * w + dj[0] * wx + dj[1] * wy + dj[2] * wz
                               + (t[0] * wxx + t[3] * wyy + t[5] * wzz
                                  + 2.0 * (t[1] * wxy + t[2] * wxz + t[4] * wyz)) / 3.0;
                    grid[((size_t)kx[a] * kdim[1] + ky[b]) * kdim[2] + kz[c]] += v;
                }
    }
}

/* Smooth-PME gather: field at the requested atoms from the grid potential psi,
 *   E_i = - sum_k grad_i W(k; r_i) psi(k). */
void orc_spme_gather(int n, const double *pos, const double *box, const int32_t *kdim, int order,
                     const double *psi, int n_out, const int32_t *out_idx, double *out)
{
    (void)n;
#pragma omp parallel for schedule(static)
    for (int o = 0; o < n_out; ++o) {
        int i = out_idx ? out_idx[o] : o;
        int kx[8], ky[8], kz[8];
        double m0[3][8], m1[3][8], m2[3][8];
        spline_axis(pos[3 * i], box[0], kdim[0], order, kx, m0[0], m1[0], m2[0]);
        spline_axis(pos[3 * i + 1], box[1], kdim[1], order, ky, m0[1], m1[1], m2[1]);
        spline_axis(pos[3 * i + 2], box[2], kdim[2], order, kz, m0[2], m1[2], m2[2]);
        double e[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < order; ++a)
            for (int b = 0; b < order; ++b)
                for (int c = 0; c < order; ++c) {
                    double p = psi[((size_t)kx[a] * kdim[1] + ky[b]) * kdim[2] + kz[c]];
                    e[0] -= m1[0][a] * m0[1][b] * m0[2][c] * p;
                    e[1] -= m0[0][a] * m1[1][b] * m0[2][c] * p;
                    e[2] -= m0[0][a] * m0[1][b] * m1[2][c] * p;
                }
        out[3 * o] = e[0];
        out[3 * o + 1] = e[1];
        out[3 * o + 2] = e[2];
    }
}

/* Count of real-space pairs 0 < |r| < rc under minimum image (unordered: each pair once). */
int64_t orc_count_pairs(int n, const double *pos, const double *box, double rc,
                        const int32_t *nc, const int32_t *cell_of, const int32_t *cell_start,
                        const int32_t *cell_atoms)
{
    int64_t cnt = 0;
#pragma omp parallel reduction(+ : cnt)
    {
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 1 ? n : 1));
#pragma omp for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) {
        int m = partners(i, n, nc, cell_of, cell_start, cell_atoms, cand);
        for (int c = 0; c < m; ++c) {
            int j = cand[c];
            if (j <= i)
                continue;
            double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                           pos[3 * i + 2] - pos[3 * j + 2]};
            min_image(d, box);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 > 0.0 && sqrt(r2) < rc)
                ++cnt;
        }
    }
    free(cand);
    }
    return cnt;
}

/* ------------------------------------------------------------------------------------------
 * Gradient of the polarization energy with respect to the atom positions.
 *
 * At the converged dipoles mu = A^-1 E_perm the energy E_pol = -1/2 C mu.E_perm is stationary in
 * mu, so (with A = alpha^-1 - T)
 *     dE_pol/dr_k = C [ -1/2 mu . (dT/dr_k) mu  -  mu . dE_perm/dr_k ].
 * Real space, per pair (r = r_i - r_j): the mutual term u = mu_i . T_ij mu_j
 * (T_ij = -B1' I + B2' r r^T, unscaled), and the two permanent terms w_ij(r) = mu_i . E_{j->i}(r)
 * and w_ji(-r) = mu_j . E_{i->j}(-r) with the pair's p-scale.  Every radial function obeys
 * dB_n'/dr = -r B_{n+1}' (the Ewald B_n by construction, the Thole-damped parts because the
 * lambdas come from one smeared charge, lambda9 included), so grad_r B_n' = -B_{n+1}' r.  Then
 *     dE_pol/dr_i = -C sum_j G_ij,   G = grad u(r) + grad w_ij(r) - (grad w_ji)(-r),
 * and dE_pol/dr_j = +C G_ij.
 * ------------------------------------------------------------------------------------------ */

/* 1 - lambda_k for k = 3, 5, 7, 9 (Thole damping of the 1/r^3 .. 105/r^9 tensors). */
static void thole_oml4(double r, double alpha_i, double alpha_j, double a_i, double a_j, double oml[4])
{
    double damp = pow(alpha_i * alpha_j, 1.0 / 6.0);
    if (damp == 0.0) {
        oml[0] = oml[1] = oml[2] = oml[3] = 0.0;
        return;
    }
    double a = a_i < a_j ? a_i : a_j;
    double u = r / damp;
    double eps = a * u * u * u;
    double e = exp(-eps);
    oml[0] = e;
    oml[1] = (1.0 + eps) * e;
    oml[2] = (1.0 + eps + 0.6 * eps * eps) * e;
    oml[3] = (1.0 + eps + (18.0 / 35.0) * eps * eps + (9.0 / 35.0) * eps * eps * eps) * e;
}

/* B1'..B4' of a pair (b[1..4]): Ewald B_n when in_cut, minus c_n (1 - s lambda) / r^(2n+1). */
static void damped_b(double r, double beta, int in_cut, double s, const double oml[4], double b[5])
{
    double eb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (in_cut) {
        double r2 = r * r;
        double g = beta > 0.0 ? 2.0 * beta / sqrt(ORC_PI) * exp(-beta * beta * r2) : 0.0;
        double t = 2.0 * beta * beta;
        eb[0] = erfc(beta * r) / r;
        eb[1] = (eb[0] + g) / r2;
        eb[2] = (3.0 * eb[1] + t * g) / r2;
        eb[3] = (5.0 * eb[2] + t * t * g) / r2;
        eb[4] = (7.0 * eb[3] + t * t * t * g) / r2;
    }
    const double c[5] = {0.0, 1.0, 3.0, 15.0, 105.0};
    double rp = r * r * r;   /* r^(2n+1) */
    b[0] = 0.0;
    for (int k = 1; k <= 4; ++k) {
        double lam = 1.0 - oml[k - 1];
        b[k] = eb[k] - c[k] * (1.0 - s * lam) / rp;
        rp *= r * r;
    }
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* grad_r of w = mu . E_mp(r), E_mp(r) the field at displacement r from a multipole (q, d, Theta):
 *   E_mp = q B1' r - B1' d + B2' (d.r) r + 1/3 B3' (Theta:rr) r - 2/3 B2' Theta r. */
static void grad_w(const double mu[3], double q, const double d[3], const double th[3][3], const double r[3],
                   const double b[5], double g[3])
{
    double mr = dot3(mu, r), dr = dot3(d, r), md = dot3(mu, d);
    double thr[3], thmu[3];
    for (int a = 0; a < 3; ++a) {
        thr[a] = th[a][0] * r[0] + th[a][1] * r[1] + th[a][2] * r[2];
        thmu[a] = th[a][0] * mu[0] + th[a][1] * mu[1] + th[a][2] * mu[2];
    }
    double thrr = dot3(thr, r), mthr = dot3(mu, thr);
    for (int a = 0; a < 3; ++a)
        g[a] = q * (b[1] * mu[a] - b[2] * mr * r[a])
               + b[2] * md * r[a]
               + b[2] * (d[a] * mr + mu[a] * dr) - b[3] * dr * mr * r[a]
               + (b[3] * (2.0 * thr[a] * mr + thrr * mu[a]) - b[4] * thrr * mr * r[a]) / 3.0
               - 2.0 * (b[2] * thmu[a] - b[3] * mthr * r[a]) / 3.0;
}

/* grad_r of u = mu_i . T(r) mu_j = -B1' mu_i.mu_j + B2' (mu_i.r)(mu_j.r). */
static void grad_u(const double mi[3], const double mj[3], const double r[3], const double b[5], double g[3])
{
    double mm = dot3(mi, mj), mir = dot3(mi, r), mjr = dot3(mj, r);
    for (int a = 0; a < 3; ++a)
        g[a] = b[2] * mm * r[a] - b[3] * mir * mjr * r[a] + b[2] * (mi[a] * mjr + mj[a] * mir);
}

static void mpole_of(int j, const double *q, const double *dip, const double *quad, double *qj, double d[3],
                     double th[3][3])
{
    *qj = q ? q[j] : 0.0;
    for (int a = 0; a < 3; ++a)
        d[a] = dip ? dip[3 * j + a] : 0.0;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
            th[a][c] = 0.0;
    if (quad) {
        const double *t = quad + 6 * j;
        th[0][0] = t[0]; th[0][1] = th[1][0] = t[1]; th[0][2] = th[2][0] = t[2];
        th[1][1] = t[3]; th[1][2] = th[2][1] = t[4]; th[2][2] = t[5];
    }
}

/* G_ij of one pair (see above); mutual = 0 leaves out u (listed pairs beyond rc). */
static void pair_grad(int i, int j, const double r[3], double rn, int in_cut, double s, double beta,
                      const double *alpha, const double *thole, const double *q, const double *dip,
                      const double *quad, const double *mu, double G[3])
{
    double oml[4], bp[5], bt[5], g[3], mr[3];
    thole_oml4(rn, alpha[i], alpha[j], thole[i], thole[j], oml);
    damped_b(rn, beta, in_cut, s, oml, bp);
    double qi, qj, di[3], dj[3], thi[3][3], thj[3][3];
    mpole_of(i, q, dip, quad, &qi, di, thi);
    mpole_of(j, q, dip, quad, &qj, dj, thj);
    G[0] = G[1] = G[2] = 0.0;
    if (in_cut) {
        damped_b(rn, beta, 1, 1.0, oml, bt);
        grad_u(mu + 3 * i, mu + 3 * j, r, bt, g);
        for (int a = 0; a < 3; ++a)
            G[a] += g[a];
    }
    grad_w(mu + 3 * i, qj, dj, thj, r, bp, g);
    for (int a = 0; a < 3; ++a)
        G[a] += g[a];
    for (int a = 0; a < 3; ++a)
        mr[a] = -r[a];
    grad_w(mu + 3 * j, qi, di, thi, mr, bp, g);
    for (int a = 0; a < 3; ++a)
        G[a] -= g[a];
}

/* out[o] = sum_j G_ij for the requested atoms (so that dE_pol,real/dr_i = -C out_i): the pairs
 * within rc from the partner search, the listed pairs at or beyond rc from the CSR (permanent
 * terms only, bare tensors with the pair's scale). */
void orc_polar_grad_real(int n, const double *pos, const double *box, double beta, double rc,
                         const double *alpha, const double *thole, const double *q, const double *dip,
                         const double *quad, const double *mu, const int32_t *sc_ptr, const int32_t *sc_j,
                         const double *sc_s, int n_out, const int32_t *out_idx, double *out,
                         const int32_t *nc, const int32_t *cell_of, const int32_t *cell_start,
                         const int32_t *cell_atoms)
{
#pragma omp parallel
    {
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 1 ? n : 1));
#pragma omp for schedule(dynamic, 8)
    for (int o = 0; o < n_out; ++o) {
        int i = out_idx ? out_idx[o] : o;
        double acc[3] = {0.0, 0.0, 0.0}, G[3];
        int m = partners(i, n, nc, cell_of, cell_start, cell_atoms, cand);
        for (int c = 0; c < m; ++c) {
            int j = cand[c];
            double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                           pos[3 * i + 2] - pos[3 * j + 2]};
            min_image(d, box);
            double r = sqrt(dot3(d, d));
            if (!(r < rc))
                continue;
            pair_grad(i, j, d, r, 1, pair_scale(i, j, sc_ptr, sc_j, sc_s), beta, alpha, thole, q, dip, quad, mu, G);
            for (int a = 0; a < 3; ++a)
                acc[a] += G[a];
        }
        if (sc_ptr)
            for (int k = sc_ptr[i]; k < sc_ptr[i + 1]; ++k) {
                int j = sc_j[k];
                double d[3] = {pos[3 * i] - pos[3 * j], pos[3 * i + 1] - pos[3 * j + 1],
                               pos[3 * i + 2] - pos[3 * j + 2]};
                min_image(d, box);
                double r = sqrt(dot3(d, d));
                if (r < rc || sc_s[k] == 1.0)
                    continue;
                pair_grad(i, j, d, r, 0, sc_s[k], beta, alpha, thole, q, dip, quad, mu, G);
                for (int a = 0; a < 3; ++a)
                    acc[a] += G[a];
            }
        for (int a = 0; a < 3; ++a)
            out[3 * o + a] = acc[a];
    }
    free(cand);
    }
}

/*
 * Smooth-PME part of the gradient.  With Q_mu the spread of the dipoles (Q_mu(k) = sum_i
 * mu_i . grad_i W(k; r_i)), Q_p that of the permanent multipoles, and psi_x = theta * Q_x the grid
 * potentials (theta symmetric), the reciprocal energy terms are mu.T_rec mu = -sum_k Q_mu psi_mu
 * and mu.E_perm,rec = -sum_k Q_mu psi_p = -sum_k Q_p psi_mu, so
 *     dE_pol,rec/dr_m = C sum_k [ dQ_mu(k)/dr_m (psi_mu + psi_p)(k) + dQ_p(k)/dr_m psi_mu(k) ],
 *     dQ_mu/dr_m,a = sum_b mu_m,b d_a d_b W,
 *     dQ_p/dr_m,a  = q_m d_a W + sum_b d_m,b d_a d_b W + 1/3 sum_bc Theta_m,bc d_a d_b d_c W.
 * out[o] = the bracket (psi_a = psi_mu + psi_p, psi_b = psi_mu).
 */
void orc_spme_grad(int n, const double *pos, const double *box, const int32_t *kdim, int order,
                   const double *psi_a, const double *psi_b, const double *mu, const double *q,
                   const double *dip, const double *quad, int n_out, const int32_t *out_idx, double *out)
{
    (void)n;
#pragma omp parallel for schedule(static)
    for (int o = 0; o < n_out; ++o) {
        int i = out_idx ? out_idx[o] : o;
        int kk[3][8];
        double m[3][4][8];   /* axis, derivative order, support point */
        for (int ax = 0; ax < 3; ++ax) {
            double len = box[ax];
            int K = kdim[ax];
            double u = K * (pos[3 * i + ax] / len);
            u -= K * floor(u / K);
            double fl = floor(u), fr = u - fl;
            for (int t = 0; t < order; ++t) {
                int k = (int)fl - t;
                kk[ax][t] = ((k % K) + K) % K;
                double sc = 1.0;
                for (int dv = 0; dv < 4; ++dv) {
                    m[ax][dv][t] = orc_bspline(order, fr + t, dv) * sc;
                    sc *= K / len;
                }
            }
        }
        double qi, di[3], th[3][3];
        mpole_of(i, q, dip, quad, &qi, di, th);
        const double *mi = mu + 3 * i;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < order; ++a)
            for (int b = 0; b < order; ++b)
                for (int c = 0; c < order; ++c) {
                    size_t idx = ((size_t)kk[0][a] * kdim[1] + kk[1][b]) * kdim[2] + kk[2][c];
                    double pa = psi_a[idx], pb = psi_b[idx];
                    int sup[3] = {a, b, c};
                    /* derivative of W of orders (dx, dy, dz) */
#define WD(dx, dy, dz) (m[0][dx][sup[0]] * m[1][dy][sup[1]] * m[2][dz][sup[2]])
                    for (int x = 0; x < 3; ++x) {
                        int e1[3] = {x == 0, x == 1, x == 2};
                        double hmu = 0.0, hd = 0.0, t3 = 0.0;
                        for (int y = 0; y < 3; ++y) {
                            int e2[3] = {e1[0] + (y == 0), e1[1] + (y == 1), e1[2] + (y == 2)};
                            double h = WD(e2[0], e2[1], e2[2]);
                            hmu += h * mi[y];
                            hd += h * di[y];
                            for (int z = 0; z < 3; ++z) {
                                int e3[3] = {e2[0] + (z == 0), e2[1] + (z == 1), e2[2] + (z == 2)};
                                t3 += th[y][z] * WD(e3[0], e3[1], e3[2]);
                            }
                        }
                        acc[x] += pa * hmu + pb * (qi * WD(e1[0], e1[1], e1[2]) + hd + t3 / 3.0);
                    }
#undef WD
                }
        for (int a = 0; a < 3; ++a)
            out[3 * o + a] = acc[a];
    }
}

#ifdef _OPENMP
#include <omp.h>
#endif
/* Threads the OpenMP loops above use. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
