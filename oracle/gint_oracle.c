/*
 * gint_oracle.c -- plain, slow, FP64 CPU definition of the real-space grid
 * integrals of NAO-based (RT-)TDDFT.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark may load it; the product path never links, calls or
 * includes anything from here, and this file includes nothing from the
 * product.
 *
 * What it computes (Gamma point, spin-unpolarised, Hartree atomic units):
 *
 *   basis   phi_mu(r) = f_{I l zeta}(|r|) Y_lm(r/|r|)
 *           (Sec. 2.1 "Real-Time Propagation", NAO decomposition equation);
 *           f is the clamped cubic spline through the caller's knot table;
 *           the radial derivative is taken from that spline and the angular
 *           one analytically (Sec. 2.3 "Ehrenfest Dynamics", remark after the
 *           Pulay-force equation).
 *   fold    phit_mu(r_g) = sum over lattice vectors T with |d| < rc of
 *           phi_mu(d), d = r_g - tau_I - T: the k = 0 case of the sums over
 *           lattice vectors in the rho(r_g) equation and in the H(k)/S(k)
 *           equations (Sec. 3.3.1 and Sec. 2.1).
 *   mesh    r_g = sum_i (n_i/N_i) a_i, dV = |det A| / (N1 N2 N3)
 *           (Sec. 3.3.1, H^loc equation: "elementary volume" of the mesh).
 *   H       H_mu,nu = dV sum_g phit_mu(r_g) V(r_g) phit_nu(r_g)
 *           (Sec. 3.3.1, H^loc_{mu nu}(R) equation, summed over R).
 *   rho     rho(r_g) = sum_{mu nu} D_mu,nu phit_mu(r_g) phit_nu(r_g)
 *           (Sec. 3.3.1, rho(r_g) equation, summed over R, R').
 *   force   E = dV sum_g V_g rho_g,
 *           dE/dR_I = -dV sum_g V_g sum_{mu in I} grad phit_mu(r_g) .
 *                     [(D + D^T) phit(r_g)]_mu
 *           (Sec. 3.3.1, F^{loc,Pulay} equation; the library returns the
 *           gradient dE/dR = -F).
 *
 * Readings of points the paper leaves open (mesh origin at the cell corner,
 * real-Ylm convention, orbital order l/zeta/m, clamped spline, strict r < rc,
 * r = 0 limits, image folding) are listed in the design notes of the
 * repository; each is implemented literally below.
 *
 * Loop orders deliberately differ from the GPU library's: H and the force
 * are parallel over atom rows (each thread owns its rows), rho over points.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define R_ZERO 1e-12 /* |d| below this is treated as the atom's own position */

/* real spherical harmonics, textbook closed forms (no Condon-Shortley phase) */
#define C00 0.28209479177387814 /* 1/(2 sqrt(pi))          */
#define C1 0.4886025119029199   /* sqrt(3/(4 pi))          */
#define C2 1.0925484305920792   /* sqrt(15/(4 pi))         */
#define C20 0.31539156525252005 /* sqrt(5/(16 pi))         */
#define C22 0.5462742152960396  /* sqrt(15/(16 pi))        */

typedef struct {
    int l, nr;
    double dr, rc;
    double *y;  /* knot values */
    double *m2; /* spline second derivatives at the knots */
} orad;

typedef struct {
    double lat[9]; /* rows a1, a2, a3 */
    double rec[9]; /* rows b_i with a_i . b_j = delta_ij */
    int grid[3];
    long ng;
    double dV;
    int natom;
    double *pos;
    int *spc;
    int nrad;
    orad *rad;
    int nspecies;
    int *sp_norb;   /* orbitals per species */
    int *sp_orb0;   /* offset into the per-species orbital tables */
    int *orb_rad;   /* radial index of each species-orbital */
    int *orb_l;
    int *orb_m;
    int *atom_orb0; /* first global orbital of each atom */
    double *atom_rc; /* largest cutoff among the atom's radials */
    int norb;
} octx;

/* ---------------------------------------------------------------------- */
/* clamped cubic spline through (i dr, y_i) with end slopes s0, sn.        */
/* Classic second-derivative (moment) formulation, Thomas algorithm.       */

static void spline_moments(int n, double h, const double *y, double s0, double sn, double *M)
{
    double *c = (double *)malloc(sizeof(double) * n);
    double *d = (double *)malloc(sizeof(double) * n);
    /* row 0: 2 M0 + M1 = 6/h ((y1-y0)/h - s0) */
    double b0 = 2.0, c0 = 1.0, r0 = 6.0 / h * ((y[1] - y[0]) / h - s0);
    c[0] = c0 / b0;
    d[0] = r0 / b0;
    for (int i = 1; i < n; ++i) {
        double a, b, cc, r;
        if (i < n - 1) {
            a = 1.0;
            b = 4.0;
            cc = 1.0;
            r = 6.0 / (h * h) * (y[i + 1] - 2.0 * y[i] + y[i - 1]);
        } else {
            a = 1.0;
            b = 2.0;
            cc = 0.0;
            r = 6.0 / h * (sn - (y[n - 1] - y[n - 2]) / h);
        }
        double den = b - a * c[i - 1];
        c[i] = cc / den;
        d[i] = (r - a * d[i - 1]) / den;
    }
    M[n - 1] = d[n - 1];
    for (int i = n - 2; i >= 0; --i)
        M[i] = d[i] - c[i] * M[i + 1];
    free(c);
    free(d);
}

/* f(r) and f'(r) of the spline; zero for r >= rc (strict cutoff). */
static double radial_eval(const orad *R, double r, double *dfdr)
{
    if (r >= R->rc) {
        if (dfdr)
            *dfdr = 0.0;
        return 0.0;
    }
    const double h = R->dr;
    int i = (int)floor(r / h);
    if (i > R->nr - 2)
        i = R->nr - 2;
    if (i < 0)
        i = 0;
    const double t = r - i * h;
    const double yi = R->y[i], yj = R->y[i + 1];
    const double Mi = R->m2[i], Mj = R->m2[i + 1];
    const double a = yi;
    const double b = (yj - yi) / h - h * (2.0 * Mi + Mj) / 6.0;
    const double c = Mi / 2.0;
    const double d = (Mj - Mi) / (6.0 * h);
    if (dfdr)
        *dfdr = b + t * (2.0 * c + t * 3.0 * d);
    return a + t * (b + t * (c + t * d));
}

/* S_lm(d) = |d|^l Y_lm(d/|d|) and its cartesian gradient, for l <= 2. */
static void solid_harmonic(int l, int m, const double *d, double *S, double *gS)
{
    const double x = d[0], y = d[1], z = d[2];
    double s = 0, g0 = 0, g1 = 0, g2 = 0;
    if (l == 0) {
        s = C00;
    } else if (l == 1) {
        if (m == -1) {
            s = C1 * y;
            g1 = C1;
        } else if (m == 0) {
            s = C1 * z;
            g2 = C1;
        } else {
            s = C1 * x;
            g0 = C1;
        }
    } else if (l == 2) {
        switch (m) {
        case -2:
            s = C2 * x * y;
            g0 = C2 * y;
            g1 = C2 * x;
            break;
        case -1:
            s = C2 * y * z;
            g1 = C2 * z;
            g2 = C2 * y;
            break;
        case 0:
            s = C20 * (2.0 * z * z - x * x - y * y);
            g0 = -2.0 * C20 * x;
            g1 = -2.0 * C20 * y;
            g2 = 4.0 * C20 * z;
            break;
        case 1:
            s = C2 * x * z;
            g0 = C2 * z;
            g2 = C2 * x;
            break;
        default:
            s = C22 * (x * x - y * y);
            g0 = 2.0 * C22 * x;
            g1 = -2.0 * C22 * y;
            break;
        }
    }
    *S = s;
    if (gS) {
        gS[0] = g0;
        gS[1] = g1;
        gS[2] = g2;
    }
}

/* Real Y_lm at a unit vector u (exported for the pins). */
void oracle_ylm(int l, const double *u, double *out)
{
    for (int m = -l; m <= l; ++m)
        solid_harmonic(l, m, u, &out[m + l], NULL);
}

/* phi = f(r) Y(d^), grad phi = f'(r) Y d^ + f(r) grad_d Y(d/|d|)        */
/* with grad Y(d/|d|) = grad S / r^l - l S d / r^(l+2).                   */
static void orbital_value(const orad *R, int m, const double *d, double *phi, double *grad)
{
    const int l = R->l;
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double fp;
    const double f = radial_eval(R, r, &fp);
    if (r < R_ZERO) {
        /* limits at the atom's own position */
        double z3[3] = {0, 0, 0};
        *phi = (l == 0) ? f * C00 : 0.0;
        if (grad) {
            grad[0] = grad[1] = grad[2] = 0.0;
            if (l == 1) {
                double S, gS[3];
                solid_harmonic(1, m, z3, &S, gS);
                grad[0] = fp * gS[0];
                grad[1] = fp * gS[1];
                grad[2] = fp * gS[2];
            }
        }
        return;
    }
    double S, gS[3];
    solid_harmonic(l, m, d, &S, gS);
    const double rl = (l == 0) ? 1.0 : (l == 1 ? r : r * r);
    const double Y = S / rl;
    *phi = f * Y;
    if (grad) {
        for (int k = 0; k < 3; ++k) {
            const double dY = gS[k] / rl - l * S * d[k] / (rl * r * r);
            grad[k] = fp * Y * d[k] / r + f * dY;
        }
    }
}

/* ---------------------------------------------------------------------- */

static void mesh_point(const octx *c, long g, double *r)
{
    const long n3 = g % c->grid[2];
    const long n2 = (g / c->grid[2]) % c->grid[1];
    const long n1 = g / ((long)c->grid[2] * c->grid[1]);
    const double s[3] = {(double)n1 / c->grid[0], (double)n2 / c->grid[1], (double)n3 / c->grid[2]};
    for (int k = 0; k < 3; ++k)
        r[k] = s[0] * c->lat[0 + k] + s[1] * c->lat[3 + k] + s[2] * c->lat[6 + k];
}

/*
 * Folded orbitals of atom I at point r: phit_mu(r) = sum_T phi_mu(r - tau_I - T)
 * over every lattice vector T with |r - tau_I - T| < rc.  The candidate range
 * of each integer n_i follows from |(b_i . d)| <= |b_i| |d| < |b_i| rc.
 * Returns the number of images inside the cutoff; writes norb(I) values
 * (and 3*norb(I) gradient components when grad != NULL), zero if none.
 */
static int atom_phi(const octx *c, int I, const double *r, double *phi, double *grad)
{
    const int s = c->spc[I];
    const int no = c->sp_norb[s];
    const int o0 = c->sp_orb0[s];
    const double rc = c->atom_rc[I];
    for (int o = 0; o < no; ++o) {
        phi[o] = 0.0;
        if (grad)
            grad[3 * o] = grad[3 * o + 1] = grad[3 * o + 2] = 0.0;
    }
    double dd[3], fr[3];
    for (int k = 0; k < 3; ++k)
        dd[k] = r[k] - c->pos[3 * I + k];
    int lo[3], hi[3];
    for (int i = 0; i < 3; ++i) {
        fr[i] = dd[0] * c->rec[3 * i] + dd[1] * c->rec[3 * i + 1] + dd[2] * c->rec[3 * i + 2];
        const double bn = sqrt(c->rec[3 * i] * c->rec[3 * i] + c->rec[3 * i + 1] * c->rec[3 * i + 1] +
                               c->rec[3 * i + 2] * c->rec[3 * i + 2]);
        lo[i] = (int)floor(fr[i] - rc * bn);
        hi[i] = (int)ceil(fr[i] + rc * bn);
    }
    int nimg = 0;
    for (int n1 = lo[0]; n1 <= hi[0]; ++n1)
        for (int n2 = lo[1]; n2 <= hi[1]; ++n2)
            for (int n3 = lo[2]; n3 <= hi[2]; ++n3) {
                double d[3];
                for (int k = 0; k < 3; ++k)
                    d[k] = dd[k] - (n1 * c->lat[k] + n2 * c->lat[3 + k] + n3 * c->lat[6 + k]);
                const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (!(sqrt(r2) < rc))
                    continue;
                ++nimg;
                for (int o = 0; o < no; ++o) {
                    const orad *R = &c->rad[c->orb_rad[o0 + o]];
                    if (!(sqrt(r2) < R->rc))
                        continue;
                    double p, g[3];
                    orbital_value(R, c->orb_m[o0 + o], d, &p, grad ? g : NULL);
                    phi[o] += p;
                    if (grad) {
                        grad[3 * o] += g[0];
                        grad[3 * o + 1] += g[1];
                        grad[3 * o + 2] += g[2];
                    }
                }
            }
    return nimg;
}

/* ---------------------------------------------------------------------- */
/* context                                                                 */

void *oracle_create(const double *lat, const int *grid, int nrad, const int *rad_l, const int *rad_nr,
                    const double *rad_dr, const double *rad_f, const double *rad_d0, const double *rad_drc,
                    int nspecies, const int *sp_rad_begin, int natom, const int *species_of_atom,
                    const double *pos)
{
    octx *c = (octx *)calloc(1, sizeof(octx));
    memcpy(c->lat, lat, sizeof(double) * 9);
    memcpy(c->grid, grid, sizeof(int) * 3);
    c->ng = (long)grid[0] * grid[1] * grid[2];
    /* reciprocal rows: B = A^{-T}, i.e. b_i = (a_j x a_k) / det */
    const double *a1 = lat, *a2 = lat + 3, *a3 = lat + 6;
    const double det = a1[0] * (a2[1] * a3[2] - a2[2] * a3[1]) - a1[1] * (a2[0] * a3[2] - a2[2] * a3[0]) +
                       a1[2] * (a2[0] * a3[1] - a2[1] * a3[0]);
    const double *A[3] = {a1, a2, a3};
    for (int i = 0; i < 3; ++i) {
        const double *u = A[(i + 1) % 3], *v = A[(i + 2) % 3];
        c->rec[3 * i + 0] = (u[1] * v[2] - u[2] * v[1]) / det;
        c->rec[3 * i + 1] = (u[2] * v[0] - u[0] * v[2]) / det;
        c->rec[3 * i + 2] = (u[0] * v[1] - u[1] * v[0]) / det;
    }
    c->dV = fabs(det) / (double)c->ng;

    c->nrad = nrad;
    c->rad = (orad *)calloc(nrad, sizeof(orad));
    long off = 0;
    for (int k = 0; k < nrad; ++k) {
        orad *R = &c->rad[k];
        R->l = rad_l[k];
        R->nr = rad_nr[k];
        R->dr = rad_dr[k];
        R->rc = (R->nr - 1) * R->dr;
        R->y = (double *)malloc(sizeof(double) * R->nr);
        R->m2 = (double *)malloc(sizeof(double) * R->nr);
        memcpy(R->y, rad_f + off, sizeof(double) * R->nr);
        spline_moments(R->nr, R->dr, R->y, rad_d0[k], rad_drc[k], R->m2);
        off += R->nr;
    }

    /* per-species orbital tables: radials in order of increasing l (stable
       for equal l, which is the zeta order), then m = -l..l. */
    c->nspecies = nspecies;
    c->sp_norb = (int *)calloc(nspecies, sizeof(int));
    c->sp_orb0 = (int *)calloc(nspecies, sizeof(int));
    int tot = 0;
    for (int s = 0; s < nspecies; ++s) {
        int n = 0;
        for (int k = sp_rad_begin[s]; k < sp_rad_begin[s + 1]; ++k)
            n += 2 * rad_l[k] + 1;
        c->sp_norb[s] = n;
        c->sp_orb0[s] = tot;
        tot += n;
    }
    c->orb_rad = (int *)malloc(sizeof(int) * (tot > 0 ? tot : 1));
    c->orb_l = (int *)malloc(sizeof(int) * (tot > 0 ? tot : 1));
    c->orb_m = (int *)malloc(sizeof(int) * (tot > 0 ? tot : 1));
    for (int s = 0; s < nspecies; ++s) {
        int o = c->sp_orb0[s];
        for (int l = 0; l <= 2; ++l)
            for (int k = sp_rad_begin[s]; k < sp_rad_begin[s + 1]; ++k) {
                if (rad_l[k] != l)
                    continue;
                for (int m = -l; m <= l; ++m) {
                    c->orb_rad[o] = k;
                    c->orb_l[o] = l;
                    c->orb_m[o] = m;
                    ++o;
                }
            }
    }

    c->natom = natom;
    c->pos = (double *)malloc(sizeof(double) * 3 * natom);
    memcpy(c->pos, pos, sizeof(double) * 3 * natom);
    c->spc = (int *)malloc(sizeof(int) * natom);
    memcpy(c->spc, species_of_atom, sizeof(int) * natom);
    c->atom_orb0 = (int *)malloc(sizeof(int) * (natom + 1));
    c->atom_rc = (double *)malloc(sizeof(double) * natom);
    int o = 0;
    for (int I = 0; I < natom; ++I) {
        const int s = c->spc[I];
        c->atom_orb0[I] = o;
        o += c->sp_norb[s];
        double rc = 0.0;
        for (int k = sp_rad_begin[s]; k < sp_rad_begin[s + 1]; ++k)
            if (c->rad[k].rc > rc)
                rc = c->rad[k].rc;
        c->atom_rc[I] = rc;
    }
    c->atom_orb0[natom] = o;
    c->norb = o;
    return c;
}

void oracle_destroy(void *p)
{
    octx *c = (octx *)p;
    if (!c)
        return;
    for (int k = 0; k < c->nrad; ++k) {
        free(c->rad[k].y);
        free(c->rad[k].m2);
    }
    free(c->rad);
    free(c->sp_norb);
    free(c->sp_orb0);
    free(c->orb_rad);
    free(c->orb_l);
    free(c->orb_m);
    free(c->pos);
    free(c->spc);
    free(c->atom_orb0);
    free(c->atom_rc);
    free(c);
}

int oracle_norb(void *p) { return ((octx *)p)->norb; }
double oracle_dV(void *p) { return ((octx *)p)->dV; }
int oracle_atom_orb0(void *p, int I) { return ((octx *)p)->atom_orb0[I]; }

/* Spline value and slope of radial k at r (exported for the pins). */
double oracle_radial(void *p, int k, double r, double *dfdr)
{
    return radial_eval(&((octx *)p)->rad[k], r, dfdr);
}

/* All folded orbitals (dense, length norb) and optionally their gradients
   (norb x 3) at an arbitrary cartesian point. */
void oracle_phi(void *p, const double *r, double *phi, double *grad)
{
    const octx *c = (const octx *)p;
    for (int I = 0; I < c->natom; ++I) {
        const int o0 = c->atom_orb0[I];
        atom_phi(c, I, r, phi + o0, grad ? grad + 3 * o0 : NULL);
    }
}

/* Number of atoms whose folded orbitals have support at r (any image inside
   its cutoff), and the sum over such atoms of their orbital counts. */
static int support_count(const octx *c, const double *r, double *scratch)
{
    int n = 0;
    for (int J = 0; J < c->natom; ++J)
        if (atom_phi(c, J, r, scratch, NULL) > 0)
            n += c->sp_norb[c->spc[J]];
    return n;
}

/* sum_g n_g and sum_g n_g^2, n_g = orbitals with support at mesh point g. */
void oracle_support_stats(void *p, double *sum_n, double *sum_n2)
{
    const octx *c = (const octx *)p;
    double s1 = 0.0, s2 = 0.0;
#pragma omp parallel reduction(+ : s1, s2)
    {
        double *scratch = (double *)malloc(sizeof(double) * 64);
#pragma omp for schedule(static)
        for (long g = 0; g < c->ng; ++g) {
            double r[3];
            mesh_point(c, g, r);
            const double n = (double)support_count(c, r, scratch);
            s1 += n;
            s2 += n * n;
        }
        free(scratch);
    }
    *sum_n = s1;
    *sum_n2 = s2;
}

/*
 * Rows of H for atoms I in [I0, I1): out is (orb rows of I0..I1-1) x norb,
 * row-major, overwritten.  The mesh sum runs over the points idx[0..npts)
 * (all points when idx == NULL).  Parallel over atoms; each thread owns its
 * rows.
 */
void oracle_H_rows(void *p, const double *V, int I0, int I1, long npts, const long *idx, double *out)
{
    const octx *c = (const octx *)p;
    const int norb = c->norb;
    const int row0 = c->atom_orb0[I0];
    memset(out, 0, sizeof(double) * (size_t)(c->atom_orb0[I1] - row0) * norb);
#pragma omp parallel
    {
        double *phiI = (double *)malloc(sizeof(double) * 64);
        double *phiJ = (double *)malloc(sizeof(double) * 64);
#pragma omp for schedule(dynamic, 1)
        for (int I = I0; I < I1; ++I) {
            const int nI = c->sp_norb[c->spc[I]];
            double *rows = out + (size_t)(c->atom_orb0[I] - row0) * norb;
            const long nq = idx ? npts : c->ng;
            for (long q = 0; q < nq; ++q) {
                const long g = idx ? idx[q] : q;
                double r[3];
                mesh_point(c, g, r);
                if (atom_phi(c, I, r, phiI, NULL) == 0)
                    continue;
                const double w = c->dV * V[g];
                for (int J = 0; J < c->natom; ++J) {
                    if (atom_phi(c, J, r, phiJ, NULL) == 0)
                        continue;
                    const int nJ = c->sp_norb[c->spc[J]];
                    const int j0 = c->atom_orb0[J];
                    for (int a = 0; a < nI; ++a) {
                        const double wa = w * phiI[a];
                        double *row = rows + (size_t)a * norb + j0;
                        for (int b = 0; b < nJ; ++b)
                            row[b] += wa * phiJ[b];
                    }
                }
            }
        }
        free(phiI);
        free(phiJ);
    }
}

/*
 * Orbitals of atom I at point r, one set per lattice vector T with
 * |r - tau_I - T| < rc (not summed): image k has lattice multiples
 * nvec[3k..3k+2] and values phi[k*norb(I) + o] (gradients with respect to r
 * in grad[3(k*norb(I) + o) ..] when grad != NULL).  At most maximg images
 * are stored; returns how many there are (the caller checks it against
 * maximg).
 */
static int atom_image_phi(const octx *c, int I, const double *r, int maximg, int *nvec, double *phi, double *grad)
{
    const int s = c->spc[I];
    const int no = c->sp_norb[s];
    const int o0 = c->sp_orb0[s];
    const double rc = c->atom_rc[I];
    double dd[3];
    for (int k = 0; k < 3; ++k)
        dd[k] = r[k] - c->pos[3 * I + k];
    int lo[3], hi[3];
    for (int i = 0; i < 3; ++i) {
        const double f = dd[0] * c->rec[3 * i] + dd[1] * c->rec[3 * i + 1] + dd[2] * c->rec[3 * i + 2];
        const double bn = sqrt(c->rec[3 * i] * c->rec[3 * i] + c->rec[3 * i + 1] * c->rec[3 * i + 1] +
                               c->rec[3 * i + 2] * c->rec[3 * i + 2]);
        lo[i] = (int)floor(f - rc * bn);
        hi[i] = (int)ceil(f + rc * bn);
    }
    int nimg = 0;
    for (int n1 = lo[0]; n1 <= hi[0]; ++n1)
        for (int n2 = lo[1]; n2 <= hi[1]; ++n2)
            for (int n3 = lo[2]; n3 <= hi[2]; ++n3) {
                double d[3];
                for (int k = 0; k < 3; ++k)
                    d[k] = dd[k] - (n1 * c->lat[k] + n2 * c->lat[3 + k] + n3 * c->lat[6 + k]);
                const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                if (!(rr < rc))
                    continue;
                if (nimg < maximg) {
                    nvec[3 * nimg] = n1;
                    nvec[3 * nimg + 1] = n2;
                    nvec[3 * nimg + 2] = n3;
                    double *ph = phi + (size_t)nimg * no;
                    for (int o = 0; o < no; ++o) {
                        const orad *R = &c->rad[c->orb_rad[o0 + o]];
                        double *gr = grad ? grad + 3 * ((size_t)nimg * no + o) : NULL;
                        ph[o] = 0.0;
                        if (gr)
                            gr[0] = gr[1] = gr[2] = 0.0;
                        if (rr < R->rc)
                            orbital_value(R, c->orb_m[o0 + o], d, &ph[o], gr);
                    }
                }
                ++nimg;
            }
    return nimg;
}

#define MAX_IMG 64

/*
 * Lattice-vector blocks of H^loc (Sec. 3.3.1, H^loc_{mu nu}(R) equation):
 *   H_mu,nu(R) = dV sum over the mesh points g of the whole crystal of
 *                phi_mu(r_g - tau_I) V(r_g) phi_nu(r_g - tau_J - R),
 * with tau the positions as given (not wrapped into the cell) and
 * R = n1 a1 + n2 a2 + n3 a3.  A crystal point is a cell point r_g shifted
 * by a lattice vector -T; V and the mesh are periodic, so the sum runs over
 * the cell's points and the images T of atom I reaching each:
 *   H_mu,nu(R) = dV sum_{g in cell} sum_T V_g phi_mu(r_g - tau_I - T)
 *                                         phi_nu(r_g - tau_J - T - R).
 * out is [nR][orb rows of I0..I1-1][norb], overwritten; R lists the nR
 * lattice multiples (n1, n2, n3); contributions to unlisted R are dropped.
 * The sum over R of H(R) is the Gamma-point H of oracle_H_rows.  Returns
 * -1 if some point sees more than MAX_IMG images of one atom, else 0.
 * Parallel over atom rows.
 */
int oracle_HR_rows(void *p, const double *V, int I0, int I1, int nR, const int *R, double *out)
{
    const octx *c = (const octx *)p;
    const int norb = c->norb;
    const int row0 = c->atom_orb0[I0];
    const size_t nrow = (size_t)(c->atom_orb0[I1] - row0);
    memset(out, 0, sizeof(double) * (size_t)nR * nrow * norb);
    int bad = 0;
#pragma omp parallel reduction(| : bad)
    {
        double *phiI = (double *)malloc(sizeof(double) * MAX_IMG * 64);
        double *phiJ = (double *)malloc(sizeof(double) * MAX_IMG * 64);
        int nI_vec[3 * MAX_IMG], nJ_vec[3 * MAX_IMG];
#pragma omp for schedule(dynamic, 1)
        for (int I = I0; I < I1; ++I) {
            const int nI = c->sp_norb[c->spc[I]];
            const size_t rI = (size_t)(c->atom_orb0[I] - row0);
            for (long g = 0; g < c->ng; ++g) {
                double r[3];
                mesh_point(c, g, r);
                const int kI = atom_image_phi(c, I, r, MAX_IMG, nI_vec, phiI, NULL);
                if (kI == 0)
                    continue;
                if (kI > MAX_IMG) {
                    bad = 1;
                    continue;
                }
                const double w = c->dV * V[g];
                for (int J = 0; J < c->natom; ++J) {
                    const int kJ = atom_image_phi(c, J, r, MAX_IMG, nJ_vec, phiJ, NULL);
                    if (kJ > MAX_IMG) {
                        bad = 1;
                        continue;
                    }
                    const int nJ = c->sp_norb[c->spc[J]];
                    const int j0 = c->atom_orb0[J];
                    /* T is image a of I; T + R is image b of J */
                    for (int a = 0; a < kI; ++a)
                        for (int b = 0; b < kJ; ++b) {
                            int ir = -1;
                            for (int q = 0; q < nR; ++q)
                                if (R[3 * q] == nJ_vec[3 * b] - nI_vec[3 * a] &&
                                    R[3 * q + 1] == nJ_vec[3 * b + 1] - nI_vec[3 * a + 1] &&
                                    R[3 * q + 2] == nJ_vec[3 * b + 2] - nI_vec[3 * a + 2]) {
                                    ir = q;
                                    break;
                                }
                            if (ir < 0)
                                continue;
                            double *blk = out + ((size_t)ir * nrow + rI) * norb + j0;
                            for (int x = 0; x < nI; ++x) {
                                const double wa = w * phiI[(size_t)a * nI + x];
                                for (int y = 0; y < nJ; ++y)
                                    blk[(size_t)x * norb + y] += wa * phiJ[(size_t)b * nJ + y];
                            }
                        }
                }
            }
        }
        free(phiI);
        free(phiJ);
    }
    return bad ? -1 : 0;
}

/*
 * Density from lattice-vector density-matrix blocks (Sec. 3.3.1, rho(r_g)
 * equation with its sums over R and R'):
 *   rho(r_g) = sum_{R, R'} sum_{mu nu} D_mu,nu(R) phi_mu(r_g - tau_I - R')
 *                                              phi_nu(r_g - tau_J - R - R'),
 * tau the positions as given.  With image T_a = R' of atom I and T_b of
 * atom J reaching r_g, the term is the block D_IJ(T_b - T_a).  DR is
 * [nR][norb][norb] for the nR lattice multiples R (blocks of unlisted R are
 * zero).  rho at mesh points idx[0..npts) (all when idx == NULL).  Returns
 * -1 if some point sees more than MAX_IMG images of one atom, else 0.
 * Parallel over points.
 */
int oracle_rhoR(void *p, int nR, const int *R, const double *DR, long npts, const long *idx, double *rho)
{
    const octx *c = (const octx *)p;
    const int norb = c->norb;
    const long nq = idx ? npts : c->ng;
    int bad = 0;
#pragma omp parallel reduction(| : bad)
    {
        /* per atom: its images at the point and their orbital values */
        int *kimg = (int *)malloc(sizeof(int) * c->natom);
        int *nvec = (int *)malloc(sizeof(int) * 3 * MAX_IMG * c->natom);
        double *ph = (double *)malloc(sizeof(double) * MAX_IMG * 64 * c->natom);
#pragma omp for schedule(dynamic, 64)
        for (long q = 0; q < nq; ++q) {
            const long g = idx ? idx[q] : q;
            double r[3];
            mesh_point(c, g, r);
            for (int I = 0; I < c->natom; ++I) {
                kimg[I] = atom_image_phi(c, I, r, MAX_IMG, nvec + 3 * MAX_IMG * I, ph + (size_t)MAX_IMG * 64 * I, NULL);
                if (kimg[I] > MAX_IMG) {
                    bad = 1;
                    kimg[I] = 0;
                }
            }
            double acc = 0.0;
            for (int I = 0; I < c->natom; ++I) {
                const int nI = c->sp_norb[c->spc[I]];
                const int i0 = c->atom_orb0[I];
                for (int J = 0; J < c->natom; ++J) {
                    const int nJ = c->sp_norb[c->spc[J]];
                    const int j0 = c->atom_orb0[J];
                    for (int a = 0; a < kimg[I]; ++a)
                        for (int b = 0; b < kimg[J]; ++b) {
                            const int *Ta = nvec + 3 * MAX_IMG * I + 3 * a;
                            const int *Tb = nvec + 3 * MAX_IMG * J + 3 * b;
                            int ir = -1;
                            for (int k = 0; k < nR; ++k)
                                if (R[3 * k] == Tb[0] - Ta[0] && R[3 * k + 1] == Tb[1] - Ta[1] &&
                                    R[3 * k + 2] == Tb[2] - Ta[2]) {
                                    ir = k;
                                    break;
                                }
                            if (ir < 0)
                                continue;
                            const double *pa = ph + (size_t)MAX_IMG * 64 * I + (size_t)a * nI;
                            const double *pb = ph + (size_t)MAX_IMG * 64 * J + (size_t)b * nJ;
                            const double *Dblk = DR + ((size_t)ir * norb + i0) * norb + j0;
                            for (int x = 0; x < nI; ++x) {
                                double t = 0.0;
                                for (int y = 0; y < nJ; ++y)
                                    t += Dblk[(size_t)x * norb + y] * pb[y];
                                acc += pa[x] * t;
                            }
                        }
                }
            }
            rho[q] = acc;
        }
        free(kimg);
        free(nvec);
        free(ph);
    }
    return bad ? -1 : 0;
}

/*
 * dE/dR for E = dV sum_g V_g rho_g with rho from lattice-vector density
 * blocks (oracle_rhoR; Sec. 3.3.1, F^{loc,Pulay} equation with its sum over
 * R): moving atom I moves all its images, so
 *   dE/dR_I = -dV sum_g V_g sum_{images a of I} sum_o grad phi_{a,o}(r_g) t_{a,o},
 *   t_a = sum_{atoms J, images c of J} [D_IJ(T_c - T_a) + D_JI(T_a - T_c)^T] phi_c,
 * D blocks of unlisted R being zero.  out is nsel x 3 for the atoms sel[];
 * the mesh sum runs over all points.  Returns -1 if some point sees more
 * than MAX_IMG images of one atom, else 0.  Parallel over the selected
 * atoms.
 */
static int find_R(int nR, const int *R, int n1, int n2, int n3)
{
    for (int k = 0; k < nR; ++k)
        if (R[3 * k] == n1 && R[3 * k + 1] == n2 && R[3 * k + 2] == n3)
            return k;
    return -1;
}

int oracle_forceR(void *p, const double *V, int nR, const int *R, const double *DR, int nsel, const int *sel,
                  double *out)
{
    const octx *c = (const octx *)p;
    const int norb = c->norb;
    int bad = 0;
#pragma omp parallel reduction(| : bad)
    {
        double *phiI = (double *)malloc(sizeof(double) * MAX_IMG * 64);
        double *gI = (double *)malloc(sizeof(double) * 3 * MAX_IMG * 64);
        double *phiJ = (double *)malloc(sizeof(double) * MAX_IMG * 64);
        double *t = (double *)malloc(sizeof(double) * 64);
        int nI_vec[3 * MAX_IMG], nJ_vec[3 * MAX_IMG];
#pragma omp for schedule(dynamic, 1)
        for (int s = 0; s < nsel; ++s) {
            const int I = sel[s];
            const int nI = c->sp_norb[c->spc[I]];
            const int i0 = c->atom_orb0[I];
            double f[3] = {0.0, 0.0, 0.0};
            for (long g = 0; g < c->ng; ++g) {
                double r[3];
                mesh_point(c, g, r);
                const int kI = atom_image_phi(c, I, r, MAX_IMG, nI_vec, phiI, gI);
                if (kI == 0)
                    continue;
                if (kI > MAX_IMG) {
                    bad = 1;
                    continue;
                }
                const double w = c->dV * V[g];
                for (int a = 0; a < kI; ++a) {
                    const int *Ta = nI_vec + 3 * a;
                    for (int x = 0; x < nI; ++x)
                        t[x] = 0.0;
                    for (int J = 0; J < c->natom; ++J) {
                        const int kJ = atom_image_phi(c, J, r, MAX_IMG, nJ_vec, phiJ, NULL);
                        if (kJ > MAX_IMG) {
                            bad = 1;
                            continue;
                        }
                        const int nJ = c->sp_norb[c->spc[J]];
                        const int j0 = c->atom_orb0[J];
                        for (int b = 0; b < kJ; ++b) {
                            const int *Tb = nJ_vec + 3 * b;
                            const double *pb = phiJ + (size_t)b * nJ;
                            const int qp = find_R(nR, R, Tb[0] - Ta[0], Tb[1] - Ta[1], Tb[2] - Ta[2]);
                            const int qn = find_R(nR, R, Ta[0] - Tb[0], Ta[1] - Tb[1], Ta[2] - Tb[2]);
                            for (int x = 0; x < nI; ++x)
                                for (int y = 0; y < nJ; ++y) {
                                    double sxy = 0.0;
                                    if (qp >= 0)
                                        sxy += DR[((size_t)qp * norb + i0 + x) * norb + j0 + y];
                                    if (qn >= 0)
                                        sxy += DR[((size_t)qn * norb + j0 + y) * norb + i0 + x];
                                    t[x] += sxy * pb[y];
                                }
                        }
                    }
                    for (int x = 0; x < nI; ++x)
                        for (int k = 0; k < 3; ++k)
                            f[k] += w * gI[3 * ((size_t)a * nI + x) + k] * t[x];
                }
            }
            out[3 * s] = -f[0];
            out[3 * s + 1] = -f[1];
            out[3 * s + 2] = -f[2];
        }
        free(phiI);
        free(gI);
        free(phiJ);
        free(t);
    }
    return bad ? -1 : 0;
}

/*
 * rho at mesh points idx[0..npts) (or at g = 0..npts-1 when idx == NULL).
 * Parallel over points.
 */
void oracle_rho(void *p, const double *D, long npts, const long *idx, double *rho)
{
    const octx *c = (const octx *)p;
    const int norb = c->norb;
#pragma omp parallel
    {
        double *phi = (double *)malloc(sizeof(double) * norb);
        int *nz = (int *)malloc(sizeof(int) * norb);
#pragma omp for schedule(dynamic, 64)
        for (long q = 0; q < npts; ++q) {
            const long g = idx ? idx[q] : q;
            double r[3];
            mesh_point(c, g, r);
            int nnz = 0;
            for (int J = 0; J < c->natom; ++J) {
                const int j0 = c->atom_orb0[J];
                if (atom_phi(c, J, r, phi + j0, NULL) == 0)
                    continue;
                for (int b = 0; b < c->sp_norb[c->spc[J]]; ++b)
                    nz[nnz++] = j0 + b;
            }
            double s = 0.0;
            for (int a = 0; a < nnz; ++a) {
                const int mu = nz[a];
                double t = 0.0;
                for (int b = 0; b < nnz; ++b)
                    t += D[(size_t)mu * norb + nz[b]] * phi[nz[b]];
                s += phi[mu] * t;
            }
            rho[q] = s;
        }
        free(phi);
        free(nz);
    }
}

/*
 * dE/dR for the atoms listed in sel[0..nsel), E = dV sum_g V_g rho_g, with
 * the mesh sum over idx[0..npts) (all points when idx == NULL).
 * out is nsel x 3.  Parallel over the selected atoms.
 */
void oracle_force(void *p, const double *V, const double *D, int nsel, const int *sel, long npts, const long *idx,
                  double *out)
{
    const octx *c = (const octx *)p;
    const int norb = c->norb;
#pragma omp parallel
    {
        double *phi = (double *)malloc(sizeof(double) * norb);
        double *gI = (double *)malloc(sizeof(double) * 3 * 64);
        double *tmp = (double *)malloc(sizeof(double) * 64);
        int *nz = (int *)malloc(sizeof(int) * norb);
#pragma omp for schedule(dynamic, 1)
        for (int q = 0; q < nsel; ++q) {
            const int I = sel[q];
            const int nI = c->sp_norb[c->spc[I]];
            const int i0 = c->atom_orb0[I];
            double acc[3] = {0.0, 0.0, 0.0};
            const long nq = idx ? npts : c->ng;
            for (long qq = 0; qq < nq; ++qq) {
                const long g = idx ? idx[qq] : qq;
                double r[3];
                mesh_point(c, g, r);
                if (atom_phi(c, I, r, tmp, gI) == 0)
                    continue;
                int nnz = 0;
                for (int J = 0; J < c->natom; ++J) {
                    const int j0 = c->atom_orb0[J];
                    if (atom_phi(c, J, r, phi + j0, NULL) == 0)
                        continue;
                    for (int b = 0; b < c->sp_norb[c->spc[J]]; ++b)
                        nz[nnz++] = j0 + b;
                }
                const double w = c->dV * V[g];
                for (int a = 0; a < nI; ++a) {
                    const int mu = i0 + a;
                    double t = 0.0;
                    for (int b = 0; b < nnz; ++b) {
                        const int nu = nz[b];
                        t += (D[(size_t)mu * norb + nu] + D[(size_t)nu * norb + mu]) * phi[nu];
                    }
                    for (int k = 0; k < 3; ++k)
                        acc[k] -= w * gI[3 * a + k] * t;
                }
            }
            out[3 * q] = acc[0];
            out[3 * q + 1] = acc[1];
            out[3 * q + 2] = acc[2];
        }
        free(phi);
        free(gI);
        free(tmp);
        free(nz);
    }
}

/*
 * Moving-basis matrix of Sec. 2.3 (Ehrenfest dynamics, D_K equation) at the
 * Gamma point, on the mesh, with an optional weight W:
 *
 *   DK_c,mu,nu = < phit_mu | W | d phit_nu / d tau_K >_c ,  K = atom of nu,
 *              = -dV sum_g W_g phit_mu(r_g) d/dr_c phit_nu(r_g),
 *
 * since an orbital centred on tau_K depends on tau_K only through
 * r - tau_K (d/dtau_K = -grad_r); the sum over R of the D_K equation at
 * k = 0 is the folded orbital.  D_K,mu,nu vanishes unless nu belongs to K,
 * so one 3 x norb x norb array holds every D_K.  W == NULL means W = 1 (the
 * plain overlap derivative: dS_mu,nu/dtau_K = D_K,nu,mu [mu in K] +
 * D_K,mu,nu [nu in K]).
 * Rows mu of atoms I0..I1-1 over the points idx[0..npts) (all when idx is
 * NULL): out[c][row][nu], c = x, y, z, rows = orbitals of I0..I1-1 in order.
 * Parallel over the row atoms; each thread owns its rows.
 */
void oracle_DK_rows(void *p, const double *W, int I0, int I1, long npts, const long *idx, double *out)
{
    const octx *c = (const octx *)p;
    const int norb = c->norb;
    const int row0 = c->atom_orb0[I0];
    const size_t nrow = (size_t)(c->atom_orb0[I1] - row0);
    memset(out, 0, sizeof(double) * 3 * nrow * norb);
#pragma omp parallel
    {
        double *phiI = (double *)malloc(sizeof(double) * 64);
        double *phiJ = (double *)malloc(sizeof(double) * 64);
        double *gJ = (double *)malloc(sizeof(double) * 3 * 64);
#pragma omp for schedule(dynamic, 1)
        for (int I = I0; I < I1; ++I) {
            const int nI = c->sp_norb[c->spc[I]];
            const size_t r0 = (size_t)(c->atom_orb0[I] - row0);
            const long nq = idx ? npts : c->ng;
            for (long q = 0; q < nq; ++q) {
                const long g = idx ? idx[q] : q;
                double r[3];
                mesh_point(c, g, r);
                if (atom_phi(c, I, r, phiI, NULL) == 0)
                    continue;
                const double w = c->dV * (W ? W[g] : 1.0);
                for (int J = 0; J < c->natom; ++J) {
                    if (atom_phi(c, J, r, phiJ, gJ) == 0)
                        continue;
                    const int nJ = c->sp_norb[c->spc[J]];
                    const int j0 = c->atom_orb0[J];
                    for (int a = 0; a < nI; ++a) {
                        const double wa = w * phiI[a];
                        for (int k = 0; k < 3; ++k) {
                            double *row = out + ((size_t)k * nrow + r0 + a) * norb + j0;
                            for (int b = 0; b < nJ; ++b)
                                row[b] -= wa * gJ[3 * b + k];
                        }
                    }
                }
            }
        }
        free(phiI);
        free(phiJ);
        free(gJ);
    }
}

/* ---------------------------------------------------------------------- */
/* Spherical-grid projector overlaps (Sec. 3.3.2, "Spherical Grid          */
/* Integration for Nonlocal Potentials"; the velocity-gauge projector      */
/* overlap of the nonlocal pseudopotential, Sec. 2.2):                     */
/*                                                                         */
/*   Q_{p,mu}(A) = < phit_mu | e^{-i A.r} | beta_p >                       */
/*              ~= sum_{i,j} W_ij phit_mu(tau_I + x_ij) e^{-i A.(tau_I + x_ij)} */
/*                 beta_p(x_ij),                                           */
/*                                                                         */
/* on the product grid centred on the projector's atom I: x_ij = r_i u_j,  */
/* r_i = rb x_i, W_ij = rb q_i r_i^2 w_j, with (u_j, w_j) the caller's     */
/* angular rule on the unit sphere, (x_i, q_i) its radial rule on [0, 1]   */
/* and rb the largest projector cutoff of atom I's species.  beta_p(x) =   */
/* b(|x|) Y_lm(x/|x|), b the clamped cubic spline of the projector table   */
/* (strict cutoff, r = 0 limits as for the orbitals); phit is the orbital  */
/* folded over lattice images; tau_I the position as given.                */
/* ---------------------------------------------------------------------- */

typedef struct {
    int nrad;
    orad *rad;
    int nspecies;
    int *sp_begin; /* projector radials of species s: sp_begin[s] .. sp_begin[s+1]-1 */
    int *sp_nproj; /* projectors per species */
    double *sp_rb; /* largest projector cutoff per species */
} oproj;

void *oracle_proj_create(int nrad, const int *rad_l, const int *rad_nr, const double *rad_dr, const double *rad_f,
                         const double *rad_d0, const double *rad_drc, int nspecies, const int *sp_rad_begin)
{
    oproj *P = (oproj *)calloc(1, sizeof(oproj));
    P->nrad = nrad;
    P->rad = (orad *)calloc(nrad > 0 ? nrad : 1, sizeof(orad));
    long off = 0;
    for (int k = 0; k < nrad; ++k) {
        orad *R = &P->rad[k];
        R->l = rad_l[k];
        R->nr = rad_nr[k];
        R->dr = rad_dr[k];
        R->rc = (R->nr - 1) * R->dr;
        R->y = (double *)malloc(sizeof(double) * R->nr);
        R->m2 = (double *)malloc(sizeof(double) * R->nr);
        memcpy(R->y, rad_f + off, sizeof(double) * R->nr);
        spline_moments(R->nr, R->dr, R->y, rad_d0[k], rad_drc[k], R->m2);
        off += R->nr;
    }
    P->nspecies = nspecies;
    P->sp_begin = (int *)malloc(sizeof(int) * (nspecies + 1));
    P->sp_nproj = (int *)calloc(nspecies, sizeof(int));
    P->sp_rb = (double *)calloc(nspecies, sizeof(double));
    memcpy(P->sp_begin, sp_rad_begin, sizeof(int) * (nspecies + 1));
    for (int s = 0; s < nspecies; ++s)
        for (int k = sp_rad_begin[s]; k < sp_rad_begin[s + 1]; ++k) {
            P->sp_nproj[s] += 2 * rad_l[k] + 1;
            if (P->rad[k].rc > P->sp_rb[s])
                P->sp_rb[s] = P->rad[k].rc;
        }
    return P;
}

void oracle_proj_destroy(void *p)
{
    oproj *P = (oproj *)p;
    if (!P)
        return;
    for (int k = 0; k < P->nrad; ++k) {
        free(P->rad[k].y);
        free(P->rad[k].m2);
    }
    free(P->rad);
    free(P->sp_begin);
    free(P->sp_nproj);
    free(P->sp_rb);
    free(P);
}

/* projectors of the atoms before I (row offset of atom I in Q) */
int oracle_proj_row0(void *pc, void *pp, int I)
{
    const octx *c = (const octx *)pc;
    const oproj *P = (const oproj *)pp;
    int n = 0;
    for (int J = 0; J < I; ++J)
        n += P->sp_nproj[c->spc[J]];
    return n;
}

/* Rows of Q for the projectors of atoms I0..I1-1 (atoms in input order,
   within an atom the projector radials by increasing l, stable, then m):
   out is (rows) x norb complex values as (re, im) pairs, overwritten.
   Parallel over the projector atoms. */
void oracle_psibeta(void *pc, void *pp, int nang, const double *ang, int nrq, const double *rq, const double *A,
                    int I0, int I1, double *out)
{
    const octx *c = (const octx *)pc;
    const oproj *P = (const oproj *)pp;
    const int norb = c->norb;
    const int row0 = oracle_proj_row0(pc, pp, I0);
    const int nrow = oracle_proj_row0(pc, pp, I1) - row0;
    memset(out, 0, sizeof(double) * 2 * (size_t)nrow * norb);
#pragma omp parallel
    {
        double *phi = (double *)malloc(sizeof(double) * (norb > 0 ? norb : 1));
        double *beta = (double *)malloc(sizeof(double) * 64);
#pragma omp for schedule(dynamic, 1)
        for (int I = I0; I < I1; ++I) {
            const int s = c->spc[I];
            const int np = P->sp_nproj[s];
            if (np == 0)
                continue;
            const double rb = P->sp_rb[s];
            double *rows = out + 2 * (size_t)(oracle_proj_row0(pc, pp, I) - row0) * norb;
            for (int i = 0; i < nrq; ++i) {
                const double r = rb * rq[2 * i];
                const double wr = rb * rq[2 * i + 1] * r * r;
                for (int j = 0; j < nang; ++j) {
                    const double x[3] = {r * ang[4 * j], r * ang[4 * j + 1], r * ang[4 * j + 2]};
                    const double W = wr * ang[4 * j + 3];
                    double pt[3];
                    for (int k = 0; k < 3; ++k)
                        pt[k] = c->pos[3 * I + k] + x[k];
                    const double th = -(A[0] * pt[0] + A[1] * pt[1] + A[2] * pt[2]);
                    const double cr = W * cos(th), ci = W * sin(th);
                    /* projectors at x, in projector order */
                    int q = 0;
                    for (int l = 0; l <= 2; ++l)
                        for (int k = P->sp_begin[s]; k < P->sp_begin[s + 1]; ++k) {
                            if (P->rad[k].l != l)
                                continue;
                            for (int m = -l; m <= l; ++m)
                                orbital_value(&P->rad[k], m, x, &beta[q++], NULL);
                        }
                    /* every folded orbital at the point (zero where no image reaches) */
                    for (int J = 0; J < c->natom; ++J)
                        (void)atom_phi(c, J, pt, phi + c->atom_orb0[J], NULL);
                    for (int a = 0; a < np; ++a) {
                        if (beta[a] == 0.0)
                            continue;
                        double *row = rows + 2 * (size_t)a * norb;
                        const double br = cr * beta[a], bi = ci * beta[a];
                        for (int mu = 0; mu < norb; ++mu) {
                            row[2 * mu] += br * phi[mu];
                            row[2 * mu + 1] += bi * phi[mu];
                        }
                    }
                }
            }
        }
        free(phi);
        free(beta);
    }
}

/* Move atoms (for finite differences and symmetry pins). */
void oracle_set_positions(void *p, const double *pos)
{
    octx *c = (octx *)p;
    memcpy(c->pos, pos, sizeof(double) * 3 * c->natom);
}

/* Threads used by the parallel loops from now on (for timing). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
