/*
 * dugks_oracle.c -- plain FP64 CPU oracle of one D2Q9 DUGKS step (T2, and the
 * three-level T3S3 of Sec. II.B.2 in t3s3_step) for the conservative
 * Allen-Cahn equation, written from the paper (arXiv 2007.07760, Sec. II).
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; the product library never touches it.
 *
 * The step takes the paper's operations in order, one full-grid pass each, with
 * every intermediate kept in its own array so that each line can be checked
 * against an equation:
 *   1. phi at cells                      Eq. (30)
 *   2. normal n and theta                Eqs. (2), (4)
 *   3. d(phi u)/dt at cells              term of Eq. (14b), backward difference
 *   4. feq and S at cells                Eq. (14)
 *   5. f, f~+ and fbar+ at cells         Eq. (9), Eq. (23) via oracle_aux_shift
 *   6. fbar at faces, t+h                Eqs. (24)-(26)
 *   7. phi, feq, S and f at faces        Eqs. (27)-(28); face S = mean of the two cells
 *   8. meso-flux and cell update         Eq. (21), update of the Eq. (15) form with dt
 * Readings of points the paper leaves open (tau = 3 M, phi = sum f, the 1/2 of
 * the Taylor term, the isotropic stencils, the upwind tie, the time
 * discretisation of d(phi u)/dt, the first state, the fifth-order stencil of
 * T2S5) are stated at the place they are used below.
 *
 * The fifth-order reconstruction (ORC_UPWIND5, for T2S5) is a reading: the
 * paper gives no stencil.  It is pinned by exactness and error identities of
 * the interpolation, not by the paper's numbers (parity with the authors'
 * stencil unpinned); no GPU kernel implements it.
 *
 * Built with -ffp-contract=off so that each expression rounds as written.
 */
#include "dugks_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 velocities and weights in the paper's order (Sec. II.B.2, after Eq. 38):
 * xi_i = sqrt(3RT) e_i with RT = 1/3, so xi_i = e_i. */
static const int EX[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
static const int EY[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
static const double WQ[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 9.0,  1.0 / 36.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 9.0,  1.0 / 36.0};
static const double RT = 1.0 / 3.0;
/* Eq. (2) is singular where grad(phi) vanishes.  Reading: n = g / |g| with
 * |g| floored at NORMAL_EPS (n = 0 where phi is exactly flat).  Where g passes
 * through zero while theta does not -- at the extrema of the small over- and
 * undershoots the schemes produce -- n follows the rounding of g, and two
 * roundings of the same arithmetic part from there on; smooth
 * regularisations of |g| remove that but move the paper's own numbers (the
 * T2S3 entries at C = 0.25 of Tables II, III, VIII, IX by up to 10 %), so
 * the plain quotient is kept. */
static const double NORMAL_EPS = 1e-12;

static double normal_denominator(double gx, double gy) {
  const double g = sqrt(gx * gx + gy * gy);
  return g > NORMAL_EPS ? g : NORMAL_EPS;
}

/* Grids below this many cells run their loops on one thread: the fork / join
 * of a parallel region costs more than their work (and every cell's value is
 * the same either way -- no loop here is a reduction). */
#define PAR_MIN_CELLS 8192L

/* Eq. (4) with phiA = 1, phiB = 0; W = +inf turns the term off. */
static double theta_of(double phi, double width) {
  const double phiA = 1.0, phiB = 0.0;
  if (!isfinite(width)) return 0.0;
  return -4.0 * (phi - phiA) * (phi - phiB) / (width * (phiA - phiB));
}

static inline int wrap(int i, int n) {
  if (i < 0) i += n;
  if (i >= n) i -= n;
  if (i < 0 || i >= n) {
    i %= n;
    if (i < 0) i += n;
  }
  return i;
}
#define IDX(nx, x, y) ((size_t)(y) * (size_t)(nx) + (size_t)(x))

int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* threads of the loops from now on (timing the oracle on one core) */
void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ---------------------------------------------------------------- velocity */
/* Analytic prescribed fields (Sec. III; Eq. 43 rotation, Eq. 45 deformation):
 *  UNIFORM       u = p0, v = p1
 *  ROTATION      u = -p0 (y - p2), v = p0 (x - p1)            (rigid rotation)
 *  SINGLE_VORTEX u = -p0 sin^2(pi X) sin(2 pi Y) cos(pi t/p1),
 *                v =  p0 sin(2 pi X) sin^2(pi Y) cos(pi t/p1),  X = x/nx, Y = y/ny
 *  DEFORMATION   u = -p0 sin(4 pi x/nx) sin(4 pi y/ny) cos(pi t/p1),
 *                v = -p0 cos(4 pi x/nx) cos(4 pi y/ny) cos(pi t/p1)      (Eq. 45)
 */
void oracle_velocity(const oracle_params *p, double x, double y, double t,
                     double *u, double *v) {
  const double *q = p->vel_param;
  switch (p->vel_kind) {
    case ORC_VEL_UNIFORM:
      *u = q[0];
      *v = q[1];
      return;
    case ORC_VEL_ROTATION:
      *u = -q[0] * (y - q[2]);
      *v = q[0] * (x - q[1]);
      return;
    case ORC_VEL_SINGLE_VORTEX: {
      double X = x / p->nx, Y = y / p->ny;
      double g = cos(M_PI * t / q[1]);
      double sx = sin(M_PI * X), sy = sin(M_PI * Y);
      *u = -q[0] * sx * sx * sin(2.0 * M_PI * Y) * g;
      *v = q[0] * sin(2.0 * M_PI * X) * sy * sy * g;
      return;
    }
    case ORC_VEL_DEFORMATION: {
      double g = cos(M_PI * t / q[1]);
      double ax = 4.0 * M_PI * x / p->nx, ay = 4.0 * M_PI * y / p->ny;
      *u = -q[0] * sin(ax) * sin(ay) * g;
      *v = -q[0] * cos(ax) * cos(ay) * g;
      return;
    }
    default:
      *u = 0.0;
      *v = 0.0;
      return;
  }
}

/* Velocity at the centre of cell (x, y). */
static void cell_velocity(const oracle_params *p, int x, int y, double t,
                          double *u, double *v) {
  if (p->vel_kind == ORC_VEL_ARRAYS) {
    *u = p->u_arr[IDX(p->nx, x, y)];
    *v = p->v_arr[IDX(p->nx, x, y)];
    return;
  }
  oracle_velocity(p, x + 0.5, y + 0.5, t, u, v);
}

/* Velocity at the centre of the face between cell (x, y) and its neighbour in
 * direction dir (0: +x, 1: +y).  Array fields: mean of the two cells. */
static void face_velocity(const oracle_params *p, int x, int y, int dir,
                          double t, double *u, double *v) {
  if (p->vel_kind == ORC_VEL_ARRAYS) {
    int x2 = dir == 0 ? wrap(x + 1, p->nx) : x;
    int y2 = dir == 1 ? wrap(y + 1, p->ny) : y;
    *u = 0.5 * (p->u_arr[IDX(p->nx, x, y)] + p->u_arr[IDX(p->nx, x2, y2)]);
    *v = 0.5 * (p->v_arr[IDX(p->nx, x, y)] + p->v_arr[IDX(p->nx, x2, y2)]);
    return;
  }
  if (dir == 0)
    oracle_velocity(p, x + 1.0, y + 0.5, t, u, v);
  else
    oracle_velocity(p, x + 0.5, y + 1.0, t, u, v);
}

/* ------------------------------------------------- isotropic differences */
/* Reading of the isotropic finite differences (Kumar 2004, cited at Eqs. 12
 * and 26; the stencils are not printed): weighted D2Q9 moments of the 3x3
 * neighbourhood,
 *   d_a f   = (1/RT)   sum_k w_k e_ka f(x + e_k)
 *   d_ab f  = (1/RT^2) sum_k w_k (e_ka e_kb - RT delta_ab) f(x + e_k).      */
static void grad_at(int nx, int ny, const double *a, int x, int y, double *gx,
                    double *gy) {
  double sx = 0.0, sy = 0.0;
  for (int k = 0; k < 9; k++) {
    double fk = a[IDX(nx, wrap(x + EX[k], nx), wrap(y + EY[k], ny))];
    sx += WQ[k] * EX[k] * fk;
    sy += WQ[k] * EY[k] * fk;
  }
  *gx = sx / RT;
  *gy = sy / RT;
}

static void hess_at(int nx, int ny, const double *a, int x, int y, double *hxx,
                    double *hxy, double *hyy) {
  double sxx = 0.0, sxy = 0.0, syy = 0.0;
  for (int k = 0; k < 9; k++) {
    double fk = a[IDX(nx, wrap(x + EX[k], nx), wrap(y + EY[k], ny))];
    sxx += WQ[k] * (EX[k] * EX[k] - RT) * fk;
    sxy += WQ[k] * (EX[k] * EY[k]) * fk;
    syy += WQ[k] * (EY[k] * EY[k] - RT) * fk;
  }
  *hxx = sxx / (RT * RT);
  *hxy = sxy / (RT * RT);
  *hyy = syy / (RT * RT);
}

/* Gradient of phi for the normal n of Eq. (2): the isotropic one above.  A
 * test-only build (-DORC_PLANT_ANISOTROPIC_NORMAL) plants the mistake the
 * paper warns against in Sec. III.A -- two-point differences along the axes,
 * whose leading error is not isotropic -- so that a test can show that its
 * run-level isotropy check fails for it; the oracle itself never defines it. */
static void normal_grad_at(int nx, int ny, const double *a, int x, int y,
                           double *gx, double *gy) {
#ifdef ORC_PLANT_ANISOTROPIC_NORMAL
  *gx = 0.5 * (a[IDX(nx, wrap(x + 1, nx), y)] - a[IDX(nx, wrap(x - 1, nx), y)]);
  *gy = 0.5 * (a[IDX(nx, x, wrap(y + 1, ny))] - a[IDX(nx, x, wrap(y - 1, ny))]);
#else
  grad_at(nx, ny, a, x, y, gx, gy);
#endif
}

void oracle_grad(int nx, int ny, const double *a, double *gx, double *gy) {
#pragma omp parallel for schedule(static) if ((long)nx * ny >= PAR_MIN_CELLS)
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++)
      grad_at(nx, ny, a, x, y, &gx[IDX(nx, x, y)], &gy[IDX(nx, x, y)]);
}

void oracle_hess(int nx, int ny, const double *a, double *hxx, double *hxy,
                 double *hyy) {
#pragma omp parallel for schedule(static) if ((long)nx * ny >= PAR_MIN_CELLS)
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++)
      hess_at(nx, ny, a, x, y, &hxx[IDX(nx, x, y)], &hxy[IDX(nx, x, y)],
              &hyy[IDX(nx, x, y)]);
}

/* ------------------------------------------------ equilibrium and source */
/* Eq. (14a): feq_i = w_i phi (1 + xi_i.u / RT)
 * Eq. (14b): S_i   = w_i theta xi_i.n + w_i xi_i.d(phi u)/dt / RT           */
void oracle_feq_source(double phi, double ux, double uy, double theta,
                       double nvx, double nvy, double jx, double jy,
                       double feq[9], double src[9]) {
  for (int i = 0; i < 9; i++) {
    double xu = EX[i] * ux + EY[i] * uy;
    double xn = EX[i] * nvx + EY[i] * nvy;
    double xj = EX[i] * jx + EY[i] * jy;
    feq[i] = WQ[i] * phi * (1.0 + xu / RT);
    src[i] = WQ[i] * theta * xn + WQ[i] * xj / RT;
  }
}

/* ------------------------------------------- auxiliary distributions */
/* With Omega = -(f - feq)/tau, the auxiliary g = f - a (Omega + S) is linear in
 * f: g = f (1 + a/tau) - (a/tau) feq - a S.  Solve it for f, then form
 * f + b (Omega + S).  (a, b) = (dt/2, dt/2) gives f~+ from f~ (Eq. 9),
 * (dt/2, h/2) gives fbar+ from f~ (Eq. 23), (h/2, 0) gives f from fbar
 * (Eq. 27). */
double oracle_aux_shift(double g, double a, double b, double feq, double src,
                        double tau) {
  double f = (g + (a / tau) * feq + a * src) / (1.0 + a / tau);
  double omega = -(f - feq) / tau;
  return f + b * (omega + src);
}

/* ------------------------------------------------- face reconstruction */
/* Derivative planes of one fbar+ plane, from the isotropic differences. */
typedef struct {
  const double *f, *gx, *gy, *hxx, *hxy, *hyy;
} deriv_planes;

/* Upwind, Eq. (26) with the 1/2 of the Taylor series restored:
 *   fbar+(p) = f(x_k) + d.G(x_k) + (1/2) d.H(x_k).d,   d = p - x_k,
 * where x_k is the centre of the cell the characteristic comes from: the
 * upstream side of the face by the sign of the normal velocity component.
 * When that component is zero the foot of the characteristic lies on the face
 * itself; the value is then the mean of the two one-sided reconstructions. */
static double taylor2(const oracle_params *p, const deriv_planes *d, int kx,
                      int ky, double px, double py) {
  double dx = px - (kx + 0.5), dy = py - (ky + 0.5);
  size_t k = IDX(p->nx, wrap(kx, p->nx), wrap(ky, p->ny));
  return d->f[k] + (dx * d->gx[k] + dy * d->gy[k]) +
         0.5 * (dx * dx * d->hxx[k] + 2.0 * dx * dy * d->hxy[k] +
                dy * dy * d->hyy[k]);
}

/* Value of plane a at cell L + s*normal + t*tangent with periodic wrap; the
 * tangent of the +x normal is +y and that of the +y normal is +x. */
static inline double at_nt(const oracle_params *p, const double *a, int x,
                           int y, int ndx, int ndy, int s, int t) {
  int tdx = ndy, tdy = ndx;
  return a[IDX(p->nx, wrap(x + s * ndx + t * tdx, p->nx),
               wrap(y + s * ndy + t * tdy, p->ny))];
}

/* Lagrange weights w[j - m0] of the nodes j = m0..m1 (unit spacing) for the
 * value at coordinate c: w_j = prod_{k != j} (c - k) / (j - k). */
static void lagrange(int m0, int m1, double c, double *w) {
  for (int j = m0; j <= m1; j++) {
    double v = 1.0;
    for (int k = m0; k <= m1; k++)
      if (k != j) v *= (c - k) / (double)(j - k);
    w[j - m0] = v;
  }
}

/* One face value bf_i for the face between L = (x, y) and R = L + (ndx, ndy). */
static double face_value(const oracle_params *p, const deriv_planes *d, int i,
                         int x, int y, int ndx, int ndy, double h) {
  const double *a = d->f;
  int en = EX[i] * ndx + EY[i] * ndy;   /* xi_i . normal  */
  int et = EX[i] * ndy + EY[i] * ndx;   /* xi_i . tangent */
  if (p->recon == ORC_UPWIND5) {
    /* T2S5 (Sec. III names a fifth-order, non-isotropic reconstruction and
     * gives no stencil; reading): fbar+ at the foot x_b - xi_i h by a
     * tensor product of one-dimensional Lagrange interpolations in cell-centre
     * coordinates measured from L.  Along the normal the foot lies at
     * 1/2 - en h: five cells centred on the upstream cell (L for en > 0, R
     * for en < 0), or, with the foot on the face (en = 0), the six cells
     * centred on the face.  Along the tangent it lies at -et h: the five
     * cells centred on the row of L, or that row alone when et = 0.  Exact
     * for polynomials of degree <= 4 in each coordinate. */
    int n0 = -2, n1 = 3;                  /* en = 0 */
    if (en > 0) n1 = 2;                   /* cells L-2 .. L+2 */
    if (en < 0) n0 = -1;                  /* cells R-2 .. R+2 */
    int t0 = et != 0 ? -2 : 0, t1 = et != 0 ? 2 : 0;
    double wn[6], wt[5];
    lagrange(n0, n1, 0.5 - en * h, wn);
    lagrange(t0, t1, -et * h, wt);
    double v = 0.0;
    for (int s = n0; s <= n1; s++) {
      double row = 0.0;
      for (int t = t0; t <= t1; t++) row += wt[t - t0] * at_nt(p, a, x, y, ndx, ndy, s, t);
      v += wn[s - n0] * row;
    }
    return v;
  }
  if (p->recon == ORC_UPWIND3) {
    /* face centre x_b and foot of the characteristic x_b - xi_i h */
    double bx = x + 0.5 + 0.5 * ndx, by = y + 0.5 + 0.5 * ndy;
    double px = bx - EX[i] * h, py = by - EY[i] * h;
    if (en > 0) return taylor2(p, d, x, y, px, py);
    if (en < 0) return taylor2(p, d, x + ndx, y + ndy, px, py);
    return 0.5 * (taylor2(p, d, x, y, px, py) +
                  taylor2(p, d, x + ndx, y + ndy, px, py));
  }
  /* Central, Eq. (25): fbar+(x_b - xi h) = fbar+(x_b) - h xi . grad fbar+(x_b),
   * value and gradient at the face estimated from the cell values around it. */
  double F, dn, dt;
  if (p->recon == ORC_CENTRAL2) {
    double fL = at_nt(p, a, x, y, ndx, ndy, 0, 0);
    double fR = at_nt(p, a, x, y, ndx, ndy, 1, 0);
    F = 0.5 * (fL + fR);
    dn = fR - fL;
    dt = 0.25 * (at_nt(p, a, x, y, ndx, ndy, 0, 1) +
                 at_nt(p, a, x, y, ndx, ndy, 1, 1) -
                 at_nt(p, a, x, y, ndx, ndy, 0, -1) -
                 at_nt(p, a, x, y, ndx, ndy, 1, -1));
  } else {
    /* fourth-order central estimates on the 4 cells LL, L, R, RR along the
     * normal (offsets -1, 0, 1, 2); tangential derivative by the 5-point
     * centred difference in each of them */
    double f[4], D[4];
    for (int s = -1; s <= 2; s++) {
      f[s + 1] = at_nt(p, a, x, y, ndx, ndy, s, 0);
      D[s + 1] = (at_nt(p, a, x, y, ndx, ndy, s, -2) -
                  8.0 * at_nt(p, a, x, y, ndx, ndy, s, -1) +
                  8.0 * at_nt(p, a, x, y, ndx, ndy, s, 1) -
                  at_nt(p, a, x, y, ndx, ndy, s, 2)) / 12.0;
    }
    F = (-f[0] + 9.0 * f[1] + 9.0 * f[2] - f[3]) / 16.0;
    dn = (f[0] - 27.0 * f[1] + 27.0 * f[2] - f[3]) / 24.0;
    dt = (-D[0] + 9.0 * D[1] + 9.0 * D[2] - D[3]) / 16.0;
  }
  return F - h * (en * dn + et * dt);
}

/* buf: 5 planes of scratch for the derivatives (upwind only); h: the time the
 * characteristic is traced back over. */
static void reconstruct_h(const oracle_params *p, const double *bfp, double h,
                          double *bf_x, double *bf_y, double *buf) {
  int nx = p->nx, ny = p->ny;
  size_t N = (size_t)nx * ny;
  for (int i = 0; i < 9; i++) {
    deriv_planes d = {bfp + i * N, NULL, NULL, NULL, NULL, NULL};
    if (p->recon == ORC_UPWIND3) {
      /* spatial derivatives of fbar+ at the cell centres */
      double *gx = buf, *gy = buf + N, *hxx = buf + 2 * N, *hxy = buf + 3 * N,
             *hyy = buf + 4 * N;
      oracle_grad(nx, ny, d.f, gx, gy);
      oracle_hess(nx, ny, d.f, hxx, hxy, hyy);
      d.gx = gx; d.gy = gy; d.hxx = hxx; d.hxy = hxy; d.hyy = hyy;
    }
#pragma omp parallel for schedule(static) if ((long)nx * ny >= PAR_MIN_CELLS)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        bf_x[i * N + IDX(nx, x, y)] = face_value(p, &d, i, x, y, 1, 0, h);
        bf_y[i * N + IDX(nx, x, y)] = face_value(p, &d, i, x, y, 0, 1, h);
      }
  }
}

static void reconstruct_buf(const oracle_params *p, const double *bfp,
                            double *bf_x, double *bf_y, double *buf) {
  reconstruct_h(p, bfp, 0.5 * p->cfl, bf_x, bf_y, buf);
}

void oracle_reconstruct(const oracle_params *p, const double *bfp,
                        double *bf_x, double *bf_y) {
  double *buf = malloc(5 * (size_t)p->nx * p->ny * sizeof(double));
  if (!buf) return;
  reconstruct_buf(p, bfp, bf_x, bf_y, buf);
  free(buf);
}

/* ---------------------------------------------------------------- step */
void oracle_phi(int nx, int ny, const double *tf, double *phi) {
  size_t N = (size_t)nx * ny;
  for (size_t c = 0; c < N; c++) {
    double s = 0.0;
    for (int i = 0; i < 9; i++) s += tf[i * N + c];
    phi[c] = s;
  }
}

double oracle_mass(int nx, int ny, const double *tf) {
  /* Neumaier-compensated sum of phi over the grid */
  size_t N = (size_t)nx * ny;
  double s = 0.0, comp = 0.0;
  for (size_t c = 0; c < N; c++) {
    double v = 0.0;
    for (int i = 0; i < 9; i++) v += tf[i * N + c];
    double t = s + v;
    if (fabs(s) >= fabs(v))
      comp += (s - t) + v;
    else
      comp += (v - t) + s;
    s = t;
  }
  return s + comp;
}

/* Work arrays of one step: every intermediate of the step gets its own plane. */
typedef struct {
  double *phi, *nvx, *nvy, *theta, *jx, *jy;     /* N each   */
  double *feq, *src, *tfp, *bfp, *bf_x, *bf_y, *fb_x, *fb_y; /* 9N each */
  double *deriv;                                  /* 5N       */
  double *block;
} workspace;

static int ws_alloc(workspace *w, size_t N) {
  w->block = malloc((6 * N + 8 * 9 * N + 5 * N) * sizeof(double));
  if (!w->block) return 1;
  double *q = w->block;
  w->phi = q; q += N;
  w->nvx = q; q += N;
  w->nvy = q; q += N;
  w->theta = q; q += N;
  w->jx = q; q += N;
  w->jy = q; q += N;
  w->feq = q; q += 9 * N;
  w->src = q; q += 9 * N;
  w->tfp = q; q += 9 * N;
  w->bfp = q; q += 9 * N;
  w->bf_x = q; q += 9 * N;
  w->bf_y = q; q += 9 * N;
  w->fb_x = q; q += 9 * N;
  w->fb_y = q; q += 9 * N;
  w->deriv = q;
  return 0;
}

static void step_ws(const oracle_params *p, long n, const double *tf,
                    const double *phi_prev, double *tf_next, double *phi_now,
                    workspace *ws) {
  const int nx = p->nx, ny = p->ny;
  const size_t N = (size_t)nx * ny;
  const double dt = p->cfl;            /* Eq. (39) with dx = sqrt(3RT) = 1 */
  const double h = 0.5 * dt;           /* half step of the face evolution  */
  const double tau = p->mobility / RT; /* reading: M_phi = tau RT          */
  const double tn = n * dt;
  double *phi = ws->phi, *nvx = ws->nvx, *nvy = ws->nvy, *theta = ws->theta;
  double *jx = ws->jx, *jy = ws->jy, *feq = ws->feq, *src = ws->src;
  double *tfp = ws->tfp, *bfp = ws->bfp, *bf_x = ws->bf_x, *bf_y = ws->bf_y;
  double *fb_x = ws->fb_x, *fb_y = ws->fb_y;

  /* 1. phi = sum_i f~_i (Eq. 30; the moments of f~ equal those of f because
   *    Omega and S carry no mass). */
  oracle_phi(nx, ny, tf, phi);

  /* 2. n = grad phi / |grad phi| (Eq. 2) with the isotropic gradient, and
   *    theta = -4 (phi - phiA)(phi - phiB) / (W (phiA - phiB)) (Eq. 4),
   *    phiA = 1, phiB = 0. */
#pragma omp parallel for schedule(static) if ((long)nx * ny >= PAR_MIN_CELLS)
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      size_t c = IDX(nx, x, y);
      double gx, gy;
      normal_grad_at(nx, ny, phi, x, y, &gx, &gy);
      theta[c] = theta_of(phi[c], p->width);
      double d = normal_denominator(gx, gy);
      nvx[c] = gx / d;
      nvy[c] = gy / d;
    }

  /* 3. d(phi u)/dt at cell centres: backward difference over the last step,
   *    zero on the first step (reading; Eq. 14b leaves it open). */
#pragma omp parallel for schedule(static) if ((long)nx * ny >= PAR_MIN_CELLS)
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      size_t c = IDX(nx, x, y);
      if (n == 0 || p->dtphiu_zero) {
        jx[c] = 0.0;
        jy[c] = 0.0;
      } else {
        double u0, v0, u1, v1;
        cell_velocity(p, x, y, tn, &u1, &v1);
        cell_velocity(p, x, y, tn - dt, &u0, &v0);
        jx[c] = (phi[c] * u1 - phi_prev[c] * u0) / dt;
        jy[c] = (phi[c] * v1 - phi_prev[c] * v0) / dt;
      }
    }

  /* 4.-5. feq, S (Eq. 14) and the cell-centred f~+ (Eq. 9), fbar+ (Eq. 23). */
#pragma omp parallel for schedule(static) if ((long)nx * ny >= PAR_MIN_CELLS)
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      size_t c = IDX(nx, x, y);
      double u, v, fe[9], sr[9];
      cell_velocity(p, x, y, tn, &u, &v);
      oracle_feq_source(phi[c], u, v, theta[c], nvx[c], nvy[c], jx[c], jy[c],
                        fe, sr);
      for (int i = 0; i < 9; i++) {
        feq[i * N + c] = fe[i];
        src[i * N + c] = sr[i];
        tfp[i * N + c] =
            oracle_aux_shift(tf[i * N + c], 0.5 * dt, 0.5 * dt, fe[i], sr[i], tau);
        bfp[i * N + c] =
            oracle_aux_shift(tf[i * N + c], 0.5 * dt, 0.5 * h, fe[i], sr[i], tau);
      }
    }

  /* 6. fbar(x_b, t + h) = fbar+(x_b - xi h, t) on every face (Eqs. 24-26). */
  reconstruct_buf(p, bfp, bf_x, bf_y, ws->deriv);

  /* 7. Face moments and original f at the face: phi_b = sum_i fbar_i (Eq. 28,
   *    reading: no weight, as in Eq. 30), feq_b from phi_b and u(x_b, t + h),
   *    S_b = mean of the two neighbour cells at t (stated with Table I),
   *    then f = 2tau/(2tau+h) fbar + h/(2tau+h) feq + tau h/(2tau+h) S (Eq. 27). */
  for (int dir = 0; dir < 2; dir++) {
    const double *bf = dir == 0 ? bf_x : bf_y;
    double *fb = dir == 0 ? fb_x : fb_y;
#pragma omp parallel for schedule(static) if ((long)nx * ny >= PAR_MIN_CELLS)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        size_t c = IDX(nx, x, y);
        size_t r = dir == 0 ? IDX(nx, wrap(x + 1, nx), y)
                            : IDX(nx, x, wrap(y + 1, ny));
        double phib = 0.0;
        for (int i = 0; i < 9; i++) phib += bf[i * N + c];
        double ub, vb;
        face_velocity(p, x, y, dir, tn + h, &ub, &vb);
        for (int i = 0; i < 9; i++) {
          double feqb = WQ[i] * phib * (1.0 + (EX[i] * ub + EY[i] * vb) / RT);
          double sb = 0.5 * (src[i * N + c] + src[i * N + r]);
          fb[i * N + c] = oracle_aux_shift(bf[i * N + c], 0.5 * h, 0.0, feqb,
                                           sb, tau);
        }
      }
  }

  /* 8. Meso-flux L(f_i) = (1/|V|) sum over faces of (xi_i . n_in) f |face|
   *    (Eq. 21, inward normals, |V| = |face| = 1) and f~^{n+1} = f~+ + dt L. */
#pragma omp parallel for schedule(static) if ((long)nx * ny >= PAR_MIN_CELLS)
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      size_t c = IDX(nx, x, y);
      size_t w = IDX(nx, wrap(x - 1, nx), y);
      size_t s = IDX(nx, x, wrap(y - 1, ny));
      for (int i = 0; i < 9; i++) {
        double L = 0.0;
        L += (-EX[i]) * fb_x[i * N + c]; /* east face,  n_in = (-1, 0) */
        L += (+EX[i]) * fb_x[i * N + w]; /* west face,  n_in = (+1, 0) */
        L += (-EY[i]) * fb_y[i * N + c]; /* north face, n_in = (0, -1) */
        L += (+EY[i]) * fb_y[i * N + s]; /* south face, n_in = (0, +1) */
        tf_next[i * N + c] = tfp[i * N + c] + dt * L;
      }
    }

  /* 9. this step's phi becomes the history for the next step's d(phi u)/dt */
  memcpy(phi_now, phi, N * sizeof(double));
}

/* ---------------------------------------------------------------- T3S3
 * DUGKS-T3S3 (Sec. II.B.2): the stored variable is f^ = f - (dt/4)(Omega + S);
 * each step reconstructs the faces twice, at t_n + dt/6 and at t_n + 3 dt/4,
 * from fbar+ built at t_n and at t' = t_n + dt/3. */

/* Normal, theta, d(phi u)/dt, feq and S at the cell centres at time t, from
 * phi at t; d(phi u)/dt = (phi u(t) - phi_ref u(t_ref)) / (t - t_ref), or 0. */
static void cell_terms(const oracle_params *p, const double *phi, double t,
                       const double *phi_ref, double t_ref, int with_j,
                       double *feq, double *src) {
  const int nx = p->nx, ny = p->ny;
  const size_t N = (size_t)nx * ny;
#pragma omp parallel for schedule(static) if ((long)nx * ny >= PAR_MIN_CELLS)
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      size_t c = IDX(nx, x, y);
      double gx, gy;
      normal_grad_at(nx, ny, phi, x, y, &gx, &gy);
      double th = theta_of(phi[c], p->width);
      double d = normal_denominator(gx, gy);
      double u, v, jx = 0.0, jy = 0.0, fe[9], sr[9];
      cell_velocity(p, x, y, t, &u, &v);
      if (with_j && !p->dtphiu_zero) {
        double u0, v0;
        cell_velocity(p, x, y, t_ref, &u0, &v0);
        jx = (phi[c] * u - phi_ref[c] * u0) / (t - t_ref);
        jy = (phi[c] * v - phi_ref[c] * v0) / (t - t_ref);
      }
      oracle_feq_source(phi[c], u, v, th, gx / d, gy / d, jx, jy, fe, sr);
      for (int i = 0; i < 9; i++) {
        feq[i * N + c] = fe[i];
        src[i * N + c] = sr[i];
      }
    }
}

/* Meso-flux of one stage: fbar(x_b, t + hs) = fbar+(x_b - xi hs, t) on every
 * face (Eqs. 24-26 with the stage's own half step hs), phi_b = sum_i fbar_i,
 * feq_b from u(x_b, t + hs), S_b = mean of the two cells' S at t, f_b from
 * Eq. 27 with hs, and L_i = sum over the faces of (xi_i . n_in) f_b (Eq. 21).
 * scratch: 4 x 9 + 5 planes. */
static void meso_flux(const oracle_params *p, const double *bfp, double hs, double t,
                      const double *src, double *L, double *scratch) {
  const int nx = p->nx, ny = p->ny;
  const size_t N = (size_t)nx * ny;
  const double tau = p->mobility / RT;
  double *bf_x = scratch, *bf_y = scratch + 9 * N;
  double *fb_x = scratch + 18 * N, *fb_y = scratch + 27 * N;
  reconstruct_h(p, bfp, hs, bf_x, bf_y, scratch + 36 * N);
  for (int dir = 0; dir < 2; dir++) {
    const double *bf = dir == 0 ? bf_x : bf_y;
    double *fb = dir == 0 ? fb_x : fb_y;
#pragma omp parallel for schedule(static) if ((long)nx * ny >= PAR_MIN_CELLS)
    for (int y = 0; y < ny; y++)
      for (int x = 0; x < nx; x++) {
        size_t c = IDX(nx, x, y);
        size_t r = dir == 0 ? IDX(nx, wrap(x + 1, nx), y) : IDX(nx, x, wrap(y + 1, ny));
        double phib = 0.0;
        for (int i = 0; i < 9; i++) phib += bf[i * N + c];
        double ub, vb;
        face_velocity(p, x, y, dir, t + hs, &ub, &vb);
        for (int i = 0; i < 9; i++) {
          double feqb = WQ[i] * phib * (1.0 + (EX[i] * ub + EY[i] * vb) / RT);
          double sb = 0.5 * (src[i * N + c] + src[i * N + r]);
          fb[i * N + c] = oracle_aux_shift(bf[i * N + c], 0.5 * hs, 0.0, feqb, sb, tau);
        }
      }
  }
#pragma omp parallel for schedule(static) if ((long)nx * ny >= PAR_MIN_CELLS)
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      size_t c = IDX(nx, x, y);
      size_t w = IDX(nx, wrap(x - 1, nx), y);
      size_t s = IDX(nx, x, wrap(y - 1, ny));
      for (int i = 0; i < 9; i++)
        L[i * N + c] = (-EX[i]) * fb_x[i * N + c] + (+EX[i]) * fb_x[i * N + w] +
                       (-EY[i]) * fb_y[i * N + c] + (+EY[i]) * fb_y[i * N + s];
    }
}

static int t3s3_step(const oracle_params *p, long n, const double *fh,
                     const double *phi_prev, double *fh_next, double *phi_now) {
  const int nx = p->nx, ny = p->ny;
  const size_t N = (size_t)nx * ny;
  const double dt = p->cfl;
  const double tau = p->mobility / RT;
  const double tn = n * dt, t1 = tn + dt / 3.0;
  /* 2 x N, 11 x 9N, 41 x N of flux scratch */
  double *blk = malloc((2 * N + 11 * 9 * N + 41 * N) * sizeof(double));
  if (!blk) return 1;
  double *phi = blk, *phi1 = phi + N;
  double *feq = phi1 + N, *src = feq + 9 * N, *bfpA = src + 9 * N, *L1 = bfpA + 9 * N;
  double *tfm = L1 + 9 * N, *feq1 = tfm + 9 * N, *src1 = feq1 + 9 * N;
  double *bfpB = src1 + 9 * N, *L2 = bfpB + 9 * N, *fn = L2 + 9 * N, *q1 = fn + 9 * N;
  double *scratch = q1 + 9 * N;

  /* (i) phi at t_n from f^ (Eq. 30a); feq and S at t_n; fbar+ with half step
   *     dt/6 from f^ (Eq. 31); faces at t_n + dt/6 and L(f*). */
  oracle_phi(nx, ny, fh, phi);
  cell_terms(p, phi, tn, phi_prev, tn - dt, n > 0, feq, src);
  for (size_t k = 0; k < 9 * N; k++) {
    bfpA[k] = oracle_aux_shift(fh[k], 0.25 * dt, dt / 12.0, feq[k], src[k], tau);
    fn[k] = oracle_aux_shift(fh[k], 0.25 * dt, 0.0, feq[k], src[k], tau);   /* Eq. 32 */
  }
  meso_flux(p, bfpA, dt / 6.0, tn, src, L1, scratch);

  /* (ii) f~+ at t_n (Eq. 33) and f~ at t' = t_n + dt/3 (Eq. 15); phi at t'
   *      (Eq. 30b); feq, S at t' with d(phi u)/dt over [t_n, t'] (reading);
   *      Omega + S at t' (Eq. 29, read with the factor 6 / (6 tau + dt)). */
  for (size_t k = 0; k < 9 * N; k++) {
    double tfp = oracle_aux_shift(fh[k], 0.25 * dt, dt / 6.0, feq[k], src[k], tau);
    tfm[k] = tfp + dt / 3.0 * L1[k];
  }
  oracle_phi(nx, ny, tfm, phi1);
  cell_terms(p, phi1, t1, phi, tn, 1, feq1, src1);
  for (size_t k = 0; k < 9 * N; k++)
    q1[k] = -6.0 / (6.0 * tau + dt) * (tfm[k] - feq1[k] - tau * src1[k]);

  /* (iii) fbar+ with half step 5 dt/12 from f~ at t' (Eq. 34); faces at
   *       t_n + 3 dt/4 and L(f**). */
  for (size_t k = 0; k < 9 * N; k++)
    bfpB[k] = oracle_aux_shift(tfm[k], dt / 6.0, 5.0 * dt / 24.0, feq1[k], src1[k], tau);
  meso_flux(p, bfpB, 5.0 * dt / 12.0, t1, src1, L2, scratch);

  /* (iv) f^ at t_{n+1} (Eq. 16) from f at t_n (Eq. 32). */
  for (size_t k = 0; k < 9 * N; k++)
    fh_next[k] = fn[k] + 0.75 * dt * q1[k] + dt / 7.0 * (3.0 * L1[k] + 4.0 * L2[k]);
  memcpy(phi_now, phi, N * sizeof(double));
  free(blk);
  return 0;
}

int oracle_step(const oracle_params *p, long n, const double *tf,
                const double *phi_prev, double *tf_next, double *phi_now) {
  if (p->scheme == ORC_T3S3) return t3s3_step(p, n, tf, phi_prev, tf_next, phi_now);
  workspace ws;
  if (ws_alloc(&ws, (size_t)p->nx * p->ny)) return 1;
  step_ws(p, n, tf, phi_prev, tf_next, phi_now, &ws);
  free(ws.block);
  return 0;
}

/* Reading of the first state: f = feq at t = 0, so Omega = 0 and the stored
 * variable is feq - a S with d(phi u)/dt = 0: a = dt/2 for f~ (T2), dt/4 for
 * f^ (T3S3). */
int oracle_init(const oracle_params *p, const double *phi0, double *tf,
                double *phi_hist) {
  const int nx = p->nx, ny = p->ny;
  const size_t N = (size_t)nx * ny;
  const double dt = p->cfl;
  const double a = p->scheme == ORC_T3S3 ? 0.25 * dt : 0.5 * dt;
#pragma omp parallel for schedule(static) if ((long)nx * ny >= PAR_MIN_CELLS)
  for (int y = 0; y < ny; y++)
    for (int x = 0; x < nx; x++) {
      size_t c = IDX(nx, x, y);
      double gx, gy;
      normal_grad_at(nx, ny, phi0, x, y, &gx, &gy);
      double theta = theta_of(phi0[c], p->width);
      double d = normal_denominator(gx, gy);
      double u, v, fe[9], sr[9];
      cell_velocity(p, x, y, 0.0, &u, &v);
      oracle_feq_source(phi0[c], u, v, theta, gx / d, gy / d, 0.0, 0.0, fe, sr);
      for (int i = 0; i < 9; i++) tf[i * N + c] = fe[i] - a * sr[i];
      phi_hist[c] = phi0[c];
    }
  return 0;
}

int oracle_run(const oracle_params *p, long n0, long nsteps, double *tf,
               double *phi_hist) {
  const size_t N = (size_t)p->nx * p->ny;
  workspace ws;
  double *tf2 = malloc(9 * N * sizeof(double));
  double *ph2 = malloc(N * sizeof(double));
  if (!tf2 || !ph2 || ws_alloc(&ws, N)) {
    free(tf2);
    free(ph2);
    return 1;
  }
  for (long k = 0; k < nsteps; k++) {
    if (p->scheme == ORC_T3S3) {
      if (t3s3_step(p, n0 + k, tf, phi_hist, tf2, ph2)) {
        free(ws.block);
        free(tf2);
        free(ph2);
        return 1;
      }
    } else {
      step_ws(p, n0 + k, tf, phi_hist, tf2, ph2, &ws);
    }
    memcpy(tf, tf2, 9 * N * sizeof(double));
    memcpy(phi_hist, ph2, N * sizeof(double));
  }
  free(ws.block);
  free(tf2);
  free(ph2);
  return 0;
}
