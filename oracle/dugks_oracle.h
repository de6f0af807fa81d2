/*
 * dugks_oracle.h -- plain FP64 CPU oracle for one D2Q9 DUGKS time step of the
 * conservative Allen-Cahn equation (Yang, Zhong & Zhuo, arXiv 2007.07760).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links or
 * calls this code; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no header, table or helper with the HIP
 * path: the velocity set, weights, stencils and update are written out here
 * again from the paper.
 *
 * Layout: every field is row-major [y][x] with x contiguous; distributions are
 * velocity-major [i][y][x] (i = 0..8 in the paper's D2Q9 order, Sec. II.B.2).
 * Cell (x, y) has its centre at (x + 1/2, y + 1/2); the domain is periodic.
 */
#ifndef DUGKS_ORACLE_H
#define DUGKS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_CENTRAL2 = 0, ORC_UPWIND3 = 1, ORC_CENTRAL4 = 2, ORC_UPWIND5 = 3 };
enum { ORC_T2 = 0, ORC_T3S3 = 1 };
enum { ORC_VEL_UNIFORM = 0, ORC_VEL_ROTATION = 1, ORC_VEL_SINGLE_VORTEX = 2,
       ORC_VEL_DEFORMATION = 3, ORC_VEL_ARRAYS = 4 };

typedef struct {
  int nx, ny;            /* cells per side, periodic                                */
  double mobility;       /* M_phi of Eq. (1); tau = M_phi / RT                       */
  double width;          /* W of Eqs. (3)-(4), cells; +inf switches theta off        */
  double cfl;            /* C of Eq. (39); dt = C because dx = sqrt(3RT) = 1        */
  int recon;             /* ORC_* reconstruction                                    */
  int vel_kind;          /* ORC_VEL_*                                               */
  double vel_param[6];   /* see oracle_velocity()                                   */
  const double *u_arr;   /* ORC_VEL_ARRAYS: cell-centred u, [y][x]                  */
  const double *v_arr;   /* ORC_VEL_ARRAYS: cell-centred v, [y][x]                  */
  int dtphiu_zero;       /* 1: drop the d(phi u)/dt part of the source (test hook)  */
  int scheme;            /* ORC_T2 (stored f~, Sec. II.B.1) or ORC_T3S3 (stored f^,
                            Sec. II.B.2)                                             */
} oracle_params;

/* Prescribed velocity at point (x, y) and time t (analytic kinds only). */
void oracle_velocity(const oracle_params *p, double x, double y, double t,
                     double *u, double *v);

/* Isotropic D2Q9-weighted gradient and Hessian of a periodic field at every
 * cell centre (the isotropic finite differences the paper takes from Kumar). */
void oracle_grad(int nx, int ny, const double *a, double *gx, double *gy);
void oracle_hess(int nx, int ny, const double *a, double *hxx, double *hxy,
                 double *hyy);

/* Equilibrium (Eq. 14a) and source (Eq. 14b) for one point: nvec is the unit
 * normal, J = d(phi u)/dt. */
void oracle_feq_source(double phi, double ux, double uy, double theta,
                       double nvx, double nvy, double jx, double jy,
                       double feq[9], double src[9]);

/* Shift between auxiliary distributions (Eq. 9, Eq. 23, Eqs. 27, 31, 34):
 * g = f - a (Omega + S) is given, the original f is recovered from it and
 * f + b (Omega + S) is returned, with Omega = -(f - feq)/tau. */
double oracle_aux_shift(double g, double a, double b, double feq, double src,
                        double tau);

/* Face reconstruction of fbar(x_b, t + h) = fbar+(x_b - xi h, t) (Eq. 24) from the
 * cell-centred fbar+ planes, on every x-face (between (x,y) and (x+1,y)) and
 * every y-face (between (x,y) and (x,y+1)).  All arrays 9 planes. */
void oracle_reconstruct(const oracle_params *p, const double *bfp,
                        double *bf_x, double *bf_y);

/* One step n -> n+1 of the plan's scheme: reads the stored distributions
 * (T2: f~^n; T3S3: f^^n) and phi^{n-1}, writes those of n+1 and phi^n. */
int oracle_step(const oracle_params *p, long n, const double *tf,
                const double *phi_prev, double *tf_next, double *phi_now);

/* Initial state from f = feq at t = 0 with d(phi u)/dt = 0: T2 f~^0 = feq -
 * (dt/2) S^0, T3S3 f^^0 = feq - (dt/4) S^0; phi_hist = phi0. */
int oracle_init(const oracle_params *p, const double *phi0, double *tf,
                double *phi_hist);

/* Steps n0 .. n0+nsteps-1 in place on (tf, phi_hist). */
int oracle_run(const oracle_params *p, long n0, long nsteps, double *tf,
               double *phi_hist);

/* phi = sum_i f~_i per cell (Eq. 30), and its compensated total. */
void oracle_phi(int nx, int ny, const double *tf, double *phi);
double oracle_mass(int nx, int ny, const double *tf);

/* Number of OpenMP threads the oracle runs on (1 without OpenMP). */
int oracle_threads(void);
void oracle_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
