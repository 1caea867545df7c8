/*
 * Plain FP64 reference solver for the 2-D isotropic elastic wave equation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is part of the oracle that checks the
 * HIP path; it shares no code with it, and nothing in the product links it.
 *
 * What it computes (paper Section 3.3.1, "Finite difference approximation"):
 *   nu u_tt = A_h u + f~      at every node not on a rigid edge,
 * stepped with the explicit central-difference (leapfrog) formula of the
 * paper's full-discrete scheme:
 *   u^{m+1} = 2 u^m - u^{m-1} + dt^2 / nu * (A_h u^m + f~^m),
 * zero initial data (paper eq. for the IBVP, homogeneous initial conditions).
 *
 * The paper cites a second-order operator built from D-, D+, D0, lambda, mu
 * but does not print it.  The reading used here: A_h is minus the gradient of
 * the discrete elastic potential energy
 *
 *   V(u) = 1/2 h^2 { sum_k w_k sum_{x-edges} [(l+2m)_{i-1/2,k} (D-x u)^2
 *                                            + m_{i-1/2,k} (D-x v)^2]
 *                  + sum_i w_i sum_{z-edges} [m_{i,k-1/2} (D-z u)^2
 *                                            + (l+2m)_{i,k-1/2} (D-z v)^2]
 *                  + sum_{i,k} w_i w_k [2 l (Dx u)(Dz v) + 2 m (Dz u)(Dx v)] }
 *
 * divided by the lumped mass h^2 w_i w_k:  A_h u = -(h^2 w_i w_k)^-1 dV/du.
 * u, v are the x and depth components, l = lambda, m = mu, half-point
 * coefficients are arithmetic means of the nodal values, w = 1/2 on the first
 * and last row/column (trapezoid weights) and 1 elsewhere, Dx/Dz are central
 * differences inside and one-sided at the ends.  Inside the grid this gives
 * D+(a D-) second-derivative terms and D0(c D0) mixed terms; the traction-free
 * condition on the top row (depth 0) is natural.  Nodes on the left, right and
 * bottom edges are either rigid (held at zero, bc = 0) or absorbing (bc = 1).
 *
 * Absorbing edges (paper eq. for the boundary condition on the artificial
 * boundary, and its discrete form in Section 3.3.1): the first-order
 * Clayton-Engquist relation  u_t = B sigma(u) n,  B = -(1/rho) (n n^T / c_p +
 * t t^T / c_s),  n the outward normal and t the tangent, replaces the wave
 * equation at every edge node (corners take the relation of their side
 * column).  sigma(u) n is formed with the normal derivative one-sided into the
 * grid and the tangential derivative central (one-sided at the ends of the
 * edge), with the node's own lambda, mu, rho.  Time: the paper's centred
 * difference u_t ~ (u^{m+1} - u^{m-1}) / (2 dt), with the node's own
 * same-component term of B_h u taken at the mean of levels m+1 and m-1.
 * (Taking it at level m, the literal explicit form, has a root of modulus
 * c dt/h + sqrt(1 + (c dt/h)^2) > 1 and diverges within a few dozen steps.)
 *
 * The gradient is accumulated edge by edge and node by node (scatter form),
 * which is the energy definition written out; no per-node closed form is used.
 *
 * Field layout: comp c (0 = x, 1 = depth), row k (depth index), column i:
 *   index ((c * nz) + k) * nx + i.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX(c, k, i) ((((size_t)(c) * nz) + (k)) * nx + (i))

static double trap_w(int j, int n) { return (j == 0 || j == n - 1) ? 0.5 : 1.0; }

/* One-sided-at-the-ends first difference at index j of a line of n points:
 * returns the two (index, coefficient) pairs; coefficients include 1/h. */
static void sbp_d1(int j, int n, double h, int* j0, double* c0, int* j1, double* c1) {
    if (j == 0) {
        *j0 = 0; *c0 = -1.0 / h; *j1 = 1; *c1 = 1.0 / h;
    } else if (j == n - 1) {
        *j0 = n - 2; *c0 = -1.0 / h; *j1 = n - 1; *c1 = 1.0 / h;
    } else {
        *j0 = j - 1; *c0 = -0.5 / h; *j1 = j + 1; *c1 = 0.5 / h;
    }
}

/* g = dV/du for the quadratic energy above (both components). */
void oracle_energy_gradient(int nx, int nz, double h, const double* lam,
                            const double* mu, const double* u, double* g) {
    memset(g, 0, sizeof(double) * 2 * (size_t)nx * nz);
    /* x-edges between (i-1,k) and (i,k), weight w_k */
    for (int k = 0; k < nz; ++k) {
        double wk = trap_w(k, nz);
        for (int i = 1; i < nx; ++i) {
            size_t p0 = (size_t)k * nx + (i - 1), p1 = (size_t)k * nx + i;
            double a_h = 0.5 * ((lam[p0] + 2 * mu[p0]) + (lam[p1] + 2 * mu[p1]));
            double m_h = 0.5 * (mu[p0] + mu[p1]);
            double dux = (u[IDX(0, k, i)] - u[IDX(0, k, i - 1)]) / h;
            double dvx = (u[IDX(1, k, i)] - u[IDX(1, k, i - 1)]) / h;
            /* d/du of 1/2 h^2 w a dux^2 = h^2 w a dux * (+-1/h) */
            double fu = h * wk * a_h * dux, fv = h * wk * m_h * dvx;
            g[IDX(0, k, i)] += fu; g[IDX(0, k, i - 1)] -= fu;
            g[IDX(1, k, i)] += fv; g[IDX(1, k, i - 1)] -= fv;
        }
    }
    /* z-edges between (i,k-1) and (i,k), weight w_i */
    for (int k = 1; k < nz; ++k) {
        for (int i = 0; i < nx; ++i) {
            double wi = trap_w(i, nx);
            size_t p0 = (size_t)(k - 1) * nx + i, p1 = (size_t)k * nx + i;
            double a_h = 0.5 * ((lam[p0] + 2 * mu[p0]) + (lam[p1] + 2 * mu[p1]));
            double m_h = 0.5 * (mu[p0] + mu[p1]);
            double duz = (u[IDX(0, k, i)] - u[IDX(0, k - 1, i)]) / h;
            double dvz = (u[IDX(1, k, i)] - u[IDX(1, k - 1, i)]) / h;
            double fu = h * wi * m_h * duz, fv = h * wi * a_h * dvz;
            g[IDX(0, k, i)] += fu; g[IDX(0, k - 1, i)] -= fu;
            g[IDX(1, k, i)] += fv; g[IDX(1, k - 1, i)] -= fv;
        }
    }
    /* mixed node terms h^2 w_i w_k [l (Dx u)(Dz v) + m (Dz u)(Dx v)] */
    for (int k = 0; k < nz; ++k) {
        for (int i = 0; i < nx; ++i) {
            double w = trap_w(i, nx) * trap_w(k, nz);
            size_t p = (size_t)k * nx + i;
            int ix0, ix1, kz0, kz1;
            double cx0, cx1, cz0, cz1;
            sbp_d1(i, nx, h, &ix0, &cx0, &ix1, &cx1);
            sbp_d1(k, nz, h, &kz0, &cz0, &kz1, &cz1);
            double dxu = cx0 * u[IDX(0, k, ix0)] + cx1 * u[IDX(0, k, ix1)];
            double dxv = cx0 * u[IDX(1, k, ix0)] + cx1 * u[IDX(1, k, ix1)];
            double dzu = cz0 * u[IDX(0, kz0, i)] + cz1 * u[IDX(0, kz1, i)];
            double dzv = cz0 * u[IDX(1, kz0, i)] + cz1 * u[IDX(1, kz1, i)];
            double s = h * h * w;
            /* l (Dx u)(Dz v): d/du via Dx u, d/dv via Dz v */
            g[IDX(0, k, ix0)] += s * lam[p] * dzv * cx0;
            g[IDX(0, k, ix1)] += s * lam[p] * dzv * cx1;
            g[IDX(1, kz0, i)] += s * lam[p] * dxu * cz0;
            g[IDX(1, kz1, i)] += s * lam[p] * dxu * cz1;
            /* m (Dz u)(Dx v): d/du via Dz u, d/dv via Dx v */
            g[IDX(0, kz0, i)] += s * mu[p] * dxv * cz0;
            g[IDX(0, kz1, i)] += s * mu[p] * dxv * cz1;
            g[IDX(1, k, ix0)] += s * mu[p] * dzu * cx0;
            g[IDX(1, k, ix1)] += s * mu[p] * dzu * cx1;
        }
    }
}

static int is_rigid(int i, int k, int nx, int nz) {
    return i == 0 || i == nx - 1 || k == nz - 1;
}

/* First derivative of component c along x (dir 0) or depth (dir 1) at node
 * (i, k): forward (+1), backward (-1) or central (0) difference, one-sided
 * at the ends of the line whatever is asked. */
static double ce_deriv(const double* u, int nx, int nz, double h, int c, int i, int k,
                       int dir, int side) {
    int n = dir == 0 ? nx : nz, j = dir == 0 ? i : k;
    int j0, j1;
    double den;
    if (side > 0 || (side == 0 && j == 0)) { j0 = j; j1 = j + 1; den = h; }
    else if (side < 0 || j == n - 1) { j0 = j - 1; j1 = j; den = h; }
    else { j0 = j - 1; j1 = j + 1; den = 2 * h; }
    if (j0 < 0 || j1 > n - 1) return 0.0;
    double a = dir == 0 ? u[IDX(c, k, j0)] : u[IDX(c, j0, i)];
    double b = dir == 0 ? u[IDX(c, k, j1)] : u[IDX(c, j1, i)];
    return (b - a) / den;
}

/* B_h u at an edge node: -(1/rho) (n n^T / c_p + t t^T / c_s) sigma(u) n.
 * rate[0..1] receives the x and depth components. */
static void ce_rate(int nx, int nz, double h, const double* rho, const double* lam,
                    const double* mu, const double* u, int i, int k, double rate[2]) {
    size_t p = (size_t)k * nx + i;
    double nxv, nzv;  /* outward normal in (x, depth) */
    int sx = 0, sz = 0;   /* difference sides for x and depth derivatives */
    if (i == 0) { nxv = -1; nzv = 0; sx = +1; }
    else if (i == nx - 1) { nxv = 1; nzv = 0; sx = -1; }
    else { nxv = 0; nzv = 1; sz = -1; }
    double ux = ce_deriv(u, nx, nz, h, 0, i, k, 0, sx);
    double vx = ce_deriv(u, nx, nz, h, 1, i, k, 0, sx);
    double uz = ce_deriv(u, nx, nz, h, 0, i, k, 1, sz);
    double vz = ce_deriv(u, nx, nz, h, 1, i, k, 1, sz);
    double l = lam[p], m = mu[p], r = rho[p];
    double sxx = (l + 2 * m) * ux + l * vz;
    double szz = (l + 2 * m) * vz + l * ux;
    double sxz = m * (uz + vx);
    double tx = sxx * nxv + sxz * nzv, tz = sxz * nxv + szz * nzv;  /* sigma n */
    double cp = sqrt((l + 2 * m) / r), cs = sqrt(m / r);
    double tnx = -nzv, tnz = nxv;                                   /* tangent */
    double tn = tx * nxv + tz * nzv, tt = tx * tnx + tz * tnz;
    rate[0] = -(tn / cp * nxv + tt / cs * tnx) / r;
    rate[1] = -(tn / cp * nzv + tt / cs * tnz) / r;
}

/* u^{m+1} at every edge node from u^m (cur) and u^{m-1} (prev), written to
 * next.  The coefficient of the node's own component in B_h is found by
 * applying the (linear) rule to a unit field at that node. */
static void ce_step(int nx, int nz, double h, double dt, const double* rho,
                    const double* lam, const double* mu, const double* cur,
                    const double* prev, double* next, double* unit) {
    for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) {
            if (!is_rigid(i, k, nx, nz)) continue;
            double rate[2];
            ce_rate(nx, nz, h, rho, lam, mu, cur, i, k, rate);
            for (int c = 0; c < 2; ++c) {
                double e[2];
                unit[IDX(c, k, i)] = 1.0;
                ce_rate(nx, nz, h, rho, lam, mu, unit, i, k, e);
                unit[IDX(c, k, i)] = 0.0;
                double d = e[c];  /* own same-component coefficient */
                double off = rate[c] - d * cur[IDX(c, k, i)];
                next[IDX(c, k, i)] = ((1.0 + dt * d) * prev[IDX(c, k, i)] + 2.0 * dt * off) /
                                     (1.0 - dt * d);
            }
        }
}

/* out = A_h u at free nodes, 0 at rigid nodes. */
void oracle_apply_operator(int nx, int nz, double h, const double* lam,
                           const double* mu, const double* u, double* out) {
    oracle_energy_gradient(nx, nz, h, lam, mu, u, out);
    for (int c = 0; c < 2; ++c)
        for (int k = 0; k < nz; ++k)
            for (int i = 0; i < nx; ++i) {
                double w = trap_w(i, nx) * trap_w(k, nz);
                out[IDX(c, k, i)] = is_rigid(i, k, nx, nz)
                                        ? 0.0
                                        : -out[IDX(c, k, i)] / (h * h * w);
            }
}

/*
 * Leapfrog solve.  Forcing is a sum of nterm separable terms, each a window
 * of nodal values W[q][c][fh][fw] placed with its corner at (fi0[q], fk0[q])
 * and scaled by the series S[q][m], m = 0..nsteps-1.  Receivers sample both
 * components at nodes (rec_i[r], rec_k[r]) for every level m = 0..nsteps:
 * traces[(m * nrec + r) * 2 + c].  u0/um1 (optional) give u^0 and u^{-1}
 * (zero when NULL); ufinal (optional) receives u^{nsteps}.  bc: 0 rigid,
 * 1 absorbing left/right/bottom edges.  Forcing windows and receivers must
 * not touch edge nodes when bc = 1 (only free nodes carry the wave equation).
 * Returns 0, or -1 on invalid arguments.
 */
int oracle_solve(int nx, int nz, double h, double dt, int nsteps,
                 const double* rho, const double* lam, const double* mu,
                 int nterm, const int* fi0, const int* fk0, int fw, int fh,
                 const double* W, const double* S,
                 int nrec, const int* rec_i, const int* rec_k, double* traces,
                 const double* u0, const double* um1, double* ufinal, int bc) {
    if (nx < 3 || nz < 3 || nsteps < 0 || h <= 0 || dt <= 0) return -1;
    if (bc != 0 && bc != 1) return -1;
    for (int q = 0; q < nterm; ++q)
        if (fi0[q] < 0 || fk0[q] < 0 || fi0[q] + fw > nx || fk0[q] + fh > nz) return -1;
    for (int r = 0; r < nrec; ++r)
        if (rec_i[r] < 0 || rec_i[r] >= nx || rec_k[r] < 0 || rec_k[r] >= nz) return -1;
    size_t n = 2 * (size_t)nx * nz;
    double* prev = (double*)calloc(n, sizeof(double));
    double* cur = (double*)calloc(n, sizeof(double));
    double* acc = (double*)malloc(n * sizeof(double));
    double* unit = (double*)calloc(n, sizeof(double));
    if (!prev || !cur || !acc || !unit) {
        free(prev); free(cur); free(acc); free(unit); return -1;
    }
    if (u0) memcpy(cur, u0, n * sizeof(double));
    if (um1) memcpy(prev, um1, n * sizeof(double));
    for (int r = 0; r < nrec; ++r)
        for (int c = 0; c < 2; ++c)
            traces[(size_t)r * 2 + c] = cur[IDX(c, rec_k[r], rec_i[r])];
    for (int m = 0; m < nsteps; ++m) {
        oracle_apply_operator(nx, nz, h, lam, mu, cur, acc);
        for (int q = 0; q < nterm; ++q) {
            double s = S[(size_t)q * nsteps + m];
            const double* Wq = W + (size_t)q * 2 * fw * fh;
            for (int c = 0; c < 2; ++c)
                for (int kk = 0; kk < fh; ++kk)
                    for (int ii = 0; ii < fw; ++ii)
                        acc[IDX(c, fk0[q] + kk, fi0[q] + ii)] +=
                            s * Wq[((size_t)c * fh + kk) * fw + ii];
        }
        /* edge nodes first: they need u^{m-1} before it is overwritten */
        if (bc == 1) ce_step(nx, nz, h, dt, rho, lam, mu, cur, prev, prev, unit);
        for (int c = 0; c < 2; ++c)
            for (int k = 0; k < nz; ++k)
                for (int i = 0; i < nx; ++i) {
                    size_t p = IDX(c, k, i);
                    if (is_rigid(i, k, nx, nz)) {
                        if (bc == 0) prev[p] = 0.0;
                        continue;
                    }
                    prev[p] = 2.0 * cur[p] - prev[p] +
                              dt * dt / rho[(size_t)k * nx + i] * acc[p];
                }
        double* t = prev; prev = cur; cur = t;
        for (int r = 0; r < nrec; ++r)
            for (int c = 0; c < 2; ++c)
                traces[((size_t)(m + 1) * nrec + r) * 2 + c] =
                    cur[IDX(c, rec_k[r], rec_i[r])];
    }
    if (ufinal) memcpy(ufinal, cur, n * sizeof(double));
    free(prev); free(cur); free(acc); free(unit);
    return 0;
}
