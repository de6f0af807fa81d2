// dugks_abi.hip -- C ABI of the DUGKS library (include/dugks.h): plan
// validation and set-up on the host, launches of the device kernels.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "dugks_common.h"
#include "dugks_kernels.h"
#include "dugks_plan.h"

using namespace dugks;

namespace {

constexpr double RT = 1.0 / 3.0;

bool finite(double v) { return isfinite(v); }

// ------------------------------------------------------------ stencils
// bf = sum over the patch of c * fbar+, for face orientation o and velocity i.
void add_tap(int recon, double (&c)[NTAP], int o, int s, int q, double v) {
  int dx = o == 0 ? s : q;
  int dy = o == 0 ? q : s;
  c[tap_index(recon, o, dx, dy)] += v;
}

// Lagrange weight of node j among the unit-spaced nodes m0..m1 for the value
// at coordinate x
double lagrange_weight(int m0, int m1, int j, double x) {
  double w = 1.0;
  for (int k = m0; k <= m1; k++)
    if (k != j) w *= (x - k) / (double)(j - k);
  return w;
}

void make_coefficients(int recon, double h, double (&coef)[2][9][NTAP]) {
  memset(coef, 0, sizeof(coef));
  for (int o = 0; o < 2; o++)
    for (int i = 0; i < 9; i++) {
      double(&c)[NTAP] = coef[o][i];
      // velocity components along the face normal (n) and tangent (t)
      const int en = o == 0 ? ex(i) : ey(i);
      const int et = o == 0 ? ey(i) : ex(i);
      auto add = [&](int s, int q, double v) { add_tap(recon, c, o, s, q, v); };
      if (recon == DUGKS_UPWIND5) {
        // fbar+ at the foot x_b - xi h: along the normal at 1/2 - en h from
        // the centre of L, through the five cells centred on the upstream
        // cell (six centred on the face when en = 0); along the tangent at
        // -et h, through five cells (one when et = 0)
        const int n0 = en < 0 ? -1 : -2, n1 = en > 0 ? 2 : 3;
        const int t0 = et != 0 ? -2 : 0, t1 = et != 0 ? 2 : 0;
        for (int sn = n0; sn <= n1; sn++)
          for (int q = t0; q <= t1; q++)
            add(sn, q, lagrange_weight(n0, n1, sn, 0.5 - en * h) *
                           lagrange_weight(t0, t1, q, -et * h));
      } else if (recon == DUGKS_UPWIND3) {
        // foot of the characteristic relative to the centre of L, (n, t)
        const double pn = 0.5 - en * h, pt = -et * h;
        auto side = [&](int ks, double wgt) {
          // f(k) + d.G + (1/2) d.H.d with G = 3 sum w_m e_m f_m and
          // H = 9 sum w_m (e_m e_m - I/3) f_m over the 3x3 patch about k
          const double dn = pn - ks, dq = pt;
          const double d2 = dn * dn + dq * dq;
          add(ks, 0, wgt);
          for (int m = 0; m < 9; m++) {
            // the lattice is symmetric under x <-> y, so e_m in (n, t) axes
            const int mn = o == 0 ? ex(m) : ey(m);
            const int mt = o == 0 ? ey(m) : ex(m);
            const double de = dn * mn + dq * mt;
            const double v = 3.0 * wq(m) * de + 4.5 * wq(m) * (de * de - d2 / 3.0);
            add(ks + mn, mt, wgt * v);
          }
        };
        if (en > 0)
          side(0, 1.0);
        else if (en < 0)
          side(1, 1.0);
        else {
          side(0, 0.5);
          side(1, 0.5);
        }
      } else if (recon == DUGKS_CENTRAL2) {
        // F = (fL + fR)/2, dn = fR - fL, dt = (fL+t + fR+t - fL-t - fR-t)/4,
        // bf = F - h (en dn + et dt)
        add(0, 0, 0.5);
        add(1, 0, 0.5);
        add(1, 0, -h * en);
        add(0, 0, h * en);
        const double q = -h * et * 0.25;
        add(0, 1, q);
        add(1, 1, q);
        add(0, -1, -q);
        add(1, -1, -q);
      } else {
        // fourth order on LL, L, R, RR (s = -1..2):
        // F = (-1, 9, 9, -1)/16, dn = (1, -27, 27, -1)/24,
        // dt = sum_s F_s D_s with D = (1, -8, 0, 8, -1)/12 across the tangent
        const double wF[4] = {-1.0 / 16, 9.0 / 16, 9.0 / 16, -1.0 / 16};
        const double wN[4] = {1.0 / 24, -27.0 / 24, 27.0 / 24, -1.0 / 24};
        const double wD[5] = {1.0 / 12, -8.0 / 12, 0.0, 8.0 / 12, -1.0 / 12};
        for (int s = -1; s <= 2; s++) {
          add(s, 0, wF[s + 1]);
          add(s, 0, -h * en * wN[s + 1]);
          if (et != 0)
            for (int q = -2; q <= 2; q++)
              if (q != 0) add(s, q, -h * et * wF[s + 1] * wD[q + 2]);
        }
      }
    }
}

// Fold the full table into the compact one (see compact_index): each entry is
// taken from the east face (o = 0) of the velocity with e = (|en|, |et|), and
// every (o, i, tap) used by the scheme must map onto it with the right sign.
// Returns false if some coefficient is not reproduced (a broken symmetry).
bool make_compact(int recon, const double (&coef)[2][9][NTAP], double (&cp)[NCOMPACT]) {
  for (int k = 0; k < NCOMPACT; k++) cp[k] = 0.0;
  const int rep[4] = {0, 3, 1, 2};   // class 2|en|+|et| -> velocity (|en|, |et|)
  for (int c = 0; c < 4; c++)
    for (int t = 0; t < ntap(recon); t++)
      if (tap_used(recon, 0, rep[c], t))
        cp[compact_index(recon, 0, rep[c], t)] = coef[0][rep[c]][t];
  for (int o = 0; o < 2; o++)
    for (int i = 0; i < 9; i++)
      for (int t = 0; t < ntap(recon); t++) {
        const double want = coef[o][i][t];
        if (!tap_used(recon, o, i, t)) {
          if (want != 0.0) return false;
          continue;
        }
        const double got = cp[compact_index(recon, o, i, t)];
        if (fabs(got - want) > 1e-14 * (1.0 + fabs(want))) return false;
      }
  return true;
}

// ------------------------------------------------------ velocity tables
// u(x, y, t) = g(t) UX(x) UY(y), v = g(t) VX(x) VY(y), tables at x = k/2.
void make_tables(dugks_plan* P) {
  const dugks_params& p = P->p;
  const int nx = p.nx, ny = p.ny;
  const double* q = p.vel_param;
  P->tabx.assign(2 * (2 * (size_t)nx + 2), 0.0);
  P->taby.assign(2 * (2 * (size_t)ny + 2), 0.0);
  double* UX = P->tabx.data();
  double* VX = UX + (2 * nx + 2);
  double* UY = P->taby.data();
  double* VY = UY + (2 * ny + 2);
  P->period = 0.0;
  for (int k = 0; k < 2 * nx + 2; k++) {
    const double x = 0.5 * k;
    switch (p.vel_kind) {
      case DUGKS_VEL_UNIFORM: UX[k] = 1.0; VX[k] = 1.0; break;
      case DUGKS_VEL_ROTATION: UX[k] = 1.0; VX[k] = q[0] * (x - q[1]); break;
      case DUGKS_VEL_SINGLE_VORTEX: {
        const double s = sin(M_PI * (x / nx));
        UX[k] = -q[0] * s * s;
        VX[k] = q[0] * sin(2.0 * M_PI * (x / nx));
        break;
      }
      case DUGKS_VEL_DEFORMATION: {
        const double ax = 4.0 * M_PI * x / nx;
        UX[k] = -q[0] * sin(ax);
        VX[k] = -q[0] * cos(ax);
        break;
      }
    }
  }
  for (int k = 0; k < 2 * ny + 2; k++) {
    const double y = 0.5 * k;
    switch (p.vel_kind) {
      case DUGKS_VEL_UNIFORM: UY[k] = q[0]; VY[k] = q[1]; break;
      case DUGKS_VEL_ROTATION: UY[k] = -q[0] * (y - q[2]); VY[k] = 1.0; break;
      case DUGKS_VEL_SINGLE_VORTEX: {
        const double s = sin(M_PI * (y / ny));
        UY[k] = sin(2.0 * M_PI * (y / ny));
        VY[k] = s * s;
        break;
      }
      case DUGKS_VEL_DEFORMATION: {
        const double ay = 4.0 * M_PI * y / ny;
        UY[k] = sin(ay);
        VY[k] = cos(ay);
        break;
      }
    }
  }
  if (p.vel_kind == DUGKS_VEL_SINGLE_VORTEX || p.vel_kind == DUGKS_VEL_DEFORMATION)
    P->period = q[1];
  if (p.vel_kind == DUGKS_VEL_ROTATION) {
    // the rotation is u = -w (y - yc): UX = 1 and the sign sits in UY
  }
}

int validate(const dugks_params* p) {
  if (!p) return DUGKS_EINVAL;
  if (p->nx < 8 || p->ny < 8 || p->nx > 65536 || p->ny > 65536) return DUGKS_EINVAL;
  if (!finite(p->mobility) || !(p->mobility > 0.0)) return DUGKS_EINVAL;
  if (isnan(p->width) || !(p->width > 0.0)) return DUGKS_EINVAL;
  if (!finite(p->cfl) || !(p->cfl > 0.0) || p->cfl > 1.0) return DUGKS_EINVAL;
  if (p->recon < 0 || p->recon > 3) return DUGKS_EINVAL;
  if (p->precision < 0 || p->precision > 1) return DUGKS_EINVAL;
  if (p->vel_kind < 0 || p->vel_kind > 4) return DUGKS_EINVAL;
  if (p->flags & ~(DUGKS_FLAG_DTPHIU_ZERO | DUGKS_FLAG_MASS_FIX)) return DUGKS_EINVAL;
  if (p->tile_rows < 0 || p->tile_rows > 65536) return DUGKS_EINVAL;
  if (p->scheme != DUGKS_T2 && p->scheme != DUGKS_T3S3) return DUGKS_EINVAL;
  // T3S3: the coefficient (12 tau - dt) of f^ in Eq. 31 must stay positive
  if (p->scheme == DUGKS_T3S3 && !(p->cfl < 12.0 * (p->mobility / RT))) return DUGKS_EINVAL;
  for (int k = 0; k < 6; k++)
    if (!finite(p->vel_param[k])) return DUGKS_EINVAL;
  if ((p->vel_kind == DUGKS_VEL_SINGLE_VORTEX || p->vel_kind == DUGKS_VEL_DEFORMATION) &&
      !(p->vel_param[1] > 0.0))
    return DUGKS_EINVAL;
  // the fifth-order reconstruction (DUGKS-T2S5) runs with the T2 time scheme
  // and the analytic velocity kinds only
  if (p->recon == DUGKS_UPWIND5 &&
      (p->scheme != DUGKS_T2 || p->vel_kind == DUGKS_VEL_ARRAYS))
    return DUGKS_EUNSUPPORTED;
  return DUGKS_OK;
}

// Default rows per wavefront.  Resident wavefronts of the step kernel on one
// MI355X: 256 CUs, each 4 SIMDs x step_waves (the register budget the kernel
// variant is built for; the LDS ring fits that many).  A wavefront marches
// seg + 4 rows of work; the launch runs in ceil(tiles / resident) rounds, so
// pick the segment that minimises rounds * (seg + 4): whole rounds, little
// halo.  Segments are whole mass groups (multiples of MASS_GROUP rows).
int default_tile_rows(const dugks_params& p, int nstrips) {
  const int per_cu = 4 * step_waves(p.precision == DUGKS_F64 ? 8 : 4, p.recon,
                                    (p.flags & DUGKS_FLAG_MASS_FIX) != 0);
  const long resident = 256L * per_cu;
  int best = 64;
  long best_cost = -1;
  for (int seg = 16; seg <= 256; seg += MASS_GROUP) {
    const long tiles = (long)nstrips * ((p.ny + seg - 1) / seg);
    const long rounds = (tiles + resident - 1) / resident;
    const long cost = rounds * (long)(std::min(seg, p.ny) + 4);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = seg;
    }
  }
  return best;
}

// ------------------------------------------------------------ launches
// fix = false leaves out the fused mass correction's reduction (tile timing:
// the header then keeps the correction the next real step applies)
template <typename T, bool MFIX, int STAGE>
int launch_stage(const dugks_plan* P, void* state, int64_t n, hipStream_t s, bool fix = true) {
  const Layout& L = P->L;
  StepArgs<T> a = step_args<T>(P, STAGE);
  StepBufs<T> q = step_bufs<T>(P, state, n);
  T* dst2 = nullptr;
  const T* aux = nullptr;
  if (STAGE == STAGE_A) {           // f^^n -> f~(t'), Q
    q.dst = at<T>(state, L.off_mid);
    dst2 = at<T>(state, L.off_q);
  } else if (STAGE == STAGE_B) {    // f~(t'), Q -> f^^{n+1}
    q.src = at<T>(state, L.off_mid);
    aux = at<T>(state, L.off_q);
    q.cf = at<T>(state, L.off_coef2);
  }
  double* part = at<double>(state, L.off_groups);
  StateHeader* hd = at<StateHeader>(state, 0);
  // blocks per XCD (see step_kernel's tile order)
  const int per = a.ileave > 1 ? a.ileave * a.clen * a.nstrips : (a.nlogical + 7) / 8;
  dim3 grid(per * 8), block(LANES);
  const bool varr = P->p.vel_kind == DUGKS_VEL_ARRAYS;
  const T* uv = varr ? at<T>(state, L.off_vel) : nullptr;
#define DUGKS_LAUNCH(RR, VA)                                                                   \
  hipLaunchKernelGGL((step_kernel<T, RR, MFIX, STAGE, VA>), grid, block, 0, s, a, n, q.src,    \
                     q.dst, dst2, aux, q.cf, q.tabx, q.taby, uv, part, hd)
  switch (P->p.recon) {
    case DUGKS_CENTRAL2:
      if (varr) DUGKS_LAUNCH(DUGKS_CENTRAL2, true); else DUGKS_LAUNCH(DUGKS_CENTRAL2, false);
      break;
    case DUGKS_UPWIND3:
      if (varr) DUGKS_LAUNCH(DUGKS_UPWIND3, true); else DUGKS_LAUNCH(DUGKS_UPWIND3, false);
      break;
    case DUGKS_CENTRAL4:
      if (varr) DUGKS_LAUNCH(DUGKS_CENTRAL4, true); else DUGKS_LAUNCH(DUGKS_CENTRAL4, false);
      break;
    default:   // upwind-5: T2, analytic velocities (validate)
      if constexpr (STAGE == STAGE_T2) DUGKS_LAUNCH(DUGKS_UPWIND5, false);
      break;
  }
#undef DUGKS_LAUNCH
  if (MFIX && fix)
    hipLaunchKernelGGL(mass_fix_strips_kernel, dim3(L.tl.nstrips), dim3(LANES), 0, s,
                       part, L.ngroups, L.tl.nstrips, at<double>(state, L.off_strips), hd,
                       (double)P->p.nx * (double)P->p.ny);
  return hip_status(hipGetLastError());
}

template <typename T>
int launch_step(const dugks_plan* P, void* state, int64_t n, hipStream_t s, bool fix = true) {
  if (P->p.scheme == DUGKS_T3S3) {
    // with the fused correction, stage A applies the pending one as it reads
    // f^^n and stage B gives the partials of f^^{n+1}: one reduction per step
    if (P->p.flags & DUGKS_FLAG_MASS_FIX) {
      int rc = launch_stage<T, true, STAGE_A>(P, state, n, s, false);
      return rc ? rc : launch_stage<T, true, STAGE_B>(P, state, n, s, fix);
    }
    int rc = launch_stage<T, false, STAGE_A>(P, state, n, s);
    return rc ? rc : launch_stage<T, false, STAGE_B>(P, state, n, s);
  }
  return (P->p.flags & DUGKS_FLAG_MASS_FIX)
             ? launch_stage<T, true, STAGE_T2>(P, state, n, s, fix)
             : launch_stage<T, false, STAGE_T2>(P, state, n, s);
}

template <typename T>
int stage_head(const dugks_plan* P) {
  const Layout& L = P->L;
  void* h = nullptr;
  if (hipHostMalloc(&h, L.off_buf[0], hipHostMallocDefault) != hipSuccess) return DUGKS_EDEVICE;
  memset(h, 0, L.off_buf[0]);
  StateHeader* hd = static_cast<StateHeader*>(h);
  hd->magic = STATE_MAGIC;
  hd->nx = P->p.nx;
  hd->ny = P->p.ny;
  hd->precision = P->p.precision;
  hd->recon = P->p.recon;
  hd->fit_max = INFINITY;
  // the device tables carry dt * alpha (Eq. 27 with the stage's half step)
  // times the stencil
  const int s0 = P->p.scheme == DUGKS_T3S3 ? STAGE_A : STAGE_T2;
  T* cf = at<T>(h, L.off_coef);
  for (int k = 0; k < NCOMPACT; k++) cf[k] = T(P->dt * P->st[s0].alpha * P->compact[k]);
  T* cf2 = at<T>(h, L.off_coef2);
  for (int k = 0; k < NCOMPACT; k++)
    cf2[k] = T(P->dt * P->st[STAGE_B].alpha * P->compact2[k]);
  T* tx = at<T>(h, L.off_tabx);
  for (size_t k = 0; k < P->tabx.size(); k++) tx[k] = T(P->tabx[k]);
  T* ty = at<T>(h, L.off_taby);
  for (size_t k = 0; k < P->taby.size(); k++) ty[k] = T(P->taby[k]);
  P->head = h;
  return DUGKS_OK;
}

template <typename T>
int do_init(const dugks_plan* P, void* state, const double* phi0, const double* uv,
            hipStream_t s) {
  const Layout& L = P->L;
  const int nx = P->p.nx, ny = P->p.ny;
  std::call_once(P->staged, [P] { P->head_rc = stage_head<T>(P); });
  if (P->head_rc) return P->head_rc;
  hipError_t e;
  if ((e = hipMemcpyAsync(state, P->head, L.off_buf[0], hipMemcpyHostToDevice, s)))
    return hip_status(e);
  InitArgs<T> a;
  a.uv = nullptr;
  if (P->p.vel_kind == DUGKS_VEL_ARRAYS) {
    const int64_t n2 = 2 * (int64_t)nx * ny;
    T* dst = at<T>(state, L.off_vel);
    hipLaunchKernelGGL((velocity_store_kernel<T>), dim3((unsigned)((n2 + 255) / 256)), dim3(256),
                       0, s, uv, dst, n2);
    a.uv = dst;
  }
  a.phi0 = phi0;
  a.buf = at<T>(state, L.off_buf[0]);
  a.tabx = at<T>(state, L.off_tabx);
  a.taby = at<T>(state, L.off_taby);
  a.tl = L.tl;
  a.shift = P->p.scheme == DUGKS_T3S3 ? 0.25 * P->dt : 0.5 * P->dt;
  a.kth = isfinite(P->p.width) ? 4.0 / P->p.width : 0.0;
  dim3 grid((nx + 255) / 256, ny), block(256);
  hipLaunchKernelGGL((init_kernel<T>), grid, block, 0, s, a);
  if ((e = hipGetLastError())) return hip_status(e);
  // M0: FP64 total of phi0 itself (not of its rounded f~)
  double* part = at<double>(state, L.off_scratch);
  StateHeader* hd = at<StateHeader>(state, 0);
  hipLaunchKernelGGL((mass_partial_kernel<double, false>), dim3(MASS_BLOCKS), dim3(MASS_THREADS),
                     0, s, phi0, L.tl, nullptr, part);
  hipLaunchKernelGGL(mass_final_kernel, dim3(1), dim3(64), 0, s, part, &hd->mass0,
                     &hd->mass_now, hd);
  return hip_status(hipGetLastError());
}

template <typename T>
int do_phi(const dugks_plan* P, const void* state, int64_t n, void* out, hipStream_t s) {
  const Layout& L = P->L;
  const int nx = P->p.nx, ny = P->p.ny;
  dim3 grid((nx + 255) / 256, ny), block(256);
  hipLaunchKernelGGL((phi_kernel<T>), grid, block, 0, s, at<T>(state, L.off_buf[n & 1]), L.tl,
                     at<StateHeader>(state, 0), static_cast<T*>(out));
  return hip_status(hipGetLastError());
}

template <typename T>
int do_export(const dugks_plan* P, const void* state, int64_t n, void* out, hipStream_t s) {
  const Layout& L = P->L;
  const int nx = P->p.nx, ny = P->p.ny;
  dim3 grid((nx + 255) / 256, ny, 9), block(256);
  hipLaunchKernelGGL((export_kernel<T>), grid, block, 0, s, at<T>(state, L.off_buf[n & 1]), L.tl,
                     at<StateHeader>(state, 0), static_cast<T*>(out));
  return hip_status(hipGetLastError());
}

template <typename T>
int do_history(const dugks_plan* P, const void* state, int64_t n, void* out, hipStream_t s) {
  const Layout& L = P->L;
  dim3 grid((P->p.nx + 255) / 256, P->p.ny), block(256);
  hipLaunchKernelGGL((history_kernel<T>), grid, block, 0, s, at<T>(state, L.off_buf[n & 1]),
                     L.tl, static_cast<T*>(out));
  return hip_status(hipGetLastError());
}

template <typename T>
int do_mass(const dugks_plan* P, void* state, int64_t n, double* out, hipStream_t s) {
  const Layout& L = P->L;
  double* part = at<double>(state, L.off_scratch);
  StateHeader* hd = at<StateHeader>(state, 0);
  hipLaunchKernelGGL((mass_partial_kernel<T, true>), dim3(MASS_BLOCKS), dim3(MASS_THREADS), 0, s,
                     at<T>(state, L.off_buf[n & 1]), L.tl, hd, part);
  hipLaunchKernelGGL(mass_final_kernel, dim3(1), dim3(64), 0, s, part, &hd->mass_now, out, hd);
  return hip_status(hipGetLastError());
}

template <typename T>
int do_correct(const dugks_plan* P, void* state, int64_t n, hipStream_t s) {
  const Layout& L = P->L;
  const int nx = P->p.nx, ny = P->p.ny;
  const StateHeader* hd = at<StateHeader>(state, 0);
  dim3 grid((nx + 255) / 256, ny), block(256);
  for (int pass = 0; pass < 2; pass++) {
    int rc = do_mass<T>(P, state, n, nullptr, s);
    if (rc) return rc;
    hipLaunchKernelGGL((mass_correct_kernel<T>), grid, block, 0, s,
                       at<T>(state, L.off_buf[n & 1]), L.tl, hd);
    if (hipGetLastError() != hipSuccess) return DUGKS_EDEVICE;
  }
  return DUGKS_OK;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

int dugks_plan_create(const dugks_params* p, dugks_plan** out) {
  if (!out) return DUGKS_EINVAL;
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  dugks_plan* P = new (std::nothrow) dugks_plan();
  if (!P) return DUGKS_ENOMEM;
  P->p = *p;
  P->L = make_layout(p->nx, p->ny, p->precision, p->scheme, p->vel_kind);
  P->dt = p->cfl;                 // Eq. (39), dx = sqrt(3RT) = 1
  P->h = 0.5 * P->dt;
  P->tau = p->mobility / RT;      // M_phi = tau RT
  const double tau = P->tau, dt = P->dt, h = P->h;
  // g+ = (tau - b)/(tau + a) g + (a + b)/(tau + a) (feq + tau S) for
  // g = f - a (Omega + S), g+ = f + b (Omega + S)
  P->cA = (2 * tau - dt) / (2 * tau + dt);     // (a, b) = (dt/2, dt/2): f~+
  P->cB = 2 * dt / (2 * tau + dt);
  P->cA2 = (2 * tau - h) / (2 * tau + dt);     // (a, b) = (dt/2, h/2): fbar+
  P->cB2 = 3 * h / (2 * tau + dt);
  P->alpha = 2 * tau / (2 * tau + h);          // Eq. (27)
  P->beta = h / (2 * tau + h);
  P->gamma = tau * h / (2 * tau + h);
  // launch kinds: T2 (f~ in, half step h), T3S3 stage A (f^ in, dt/6), stage B
  // (f~ at t + dt/3 in, 5 dt/12); the shift identity above gives cbar with
  // a = the input's shift and b = half of the stage's half step
  auto stage = [&](int k, double hs, double a_in, double kap, double wo1, double wo2,
                   double toff, double troff, double jdt, int jfirst) {
    dugks_plan::StageCoef& c = P->st[k];
    c.h = hs;
    c.cbar = (a_in + 0.5 * hs) / (tau + a_in);
    c.kap = kap;
    c.wo1 = wo1;
    c.wo2 = wo2;
    c.alpha = 2 * tau / (2 * tau + hs);
    c.beta = hs / (2 * tau + hs);
    c.gamma = tau * hs / (2 * tau + hs);
    c.toff = toff;
    c.troff = troff;
    c.jdt = jdt;
    c.jfirst = jfirst;
  };
  // T2: f~+ = fbar+ + kap (X - fbar+), kap = cbar / (3 (1 - cbar))
  stage(STAGE_T2, h, 0.5 * dt, P->cB2 / (3.0 * (1.0 - P->cB2)), 1.0, 0.0, 0.0, -dt, dt, 1);
  P->st[STAGE_T2].cbar = P->cB2;   // the same value, rounded as Eq. 23's 3h / (2 tau + dt)
  {
    // stage A: cbar = 4 dt / (12 tau + 3 dt) (Eq. 31); f~+ (Eq. 33) and f^n
    // (Eq. 32) are fbar+ -/+ (cbar / (4 (1 - cbar))) (X - fbar+)
    const double c1 = (0.25 * dt + dt / 12.0) / (tau + 0.25 * dt);
    stage(STAGE_A, dt / 6.0, 0.25 * dt, c1 / (4.0 * (1.0 - c1)), 1.0 / 3.0, 3.0 / 7.0, 0.0, -dt,
          dt, 1);
    // stage B: cbar = 9 dt / (24 tau + 4 dt) (Eq. 34); (3/4) dt (Omega + S)(t')
    // = (3/4) dt 6 / ((6 tau + dt)(1 - cbar)) (X' - fbar+) (Eq. 29)
    const double c2 = (dt / 6.0 + 5.0 * dt / 24.0) / (tau + dt / 6.0);
    stage(STAGE_B, 5.0 * dt / 12.0, dt / 6.0,
          0.75 * dt * 6.0 / ((6.0 * tau + dt) * (1.0 - c2)), 4.0 / 7.0, 0.0, dt / 3.0, 0.0,
          dt / 3.0, 0);
  }
  const bool t3 = p->scheme == DUGKS_T3S3;
  make_coefficients(p->recon, t3 ? P->st[STAGE_A].h : h, P->coef);
  if (!make_compact(p->recon, P->coef, P->compact)) {
    delete P;
    return DUGKS_EINVAL;   // cannot happen for the schemes built in
  }
  if (t3) {
    double coef2[2][9][NTAP];
    make_coefficients(p->recon, P->st[STAGE_B].h, coef2);
    if (!make_compact(p->recon, coef2, P->compact2)) {
      delete P;
      return DUGKS_EINVAL;
    }
  }
  make_tables(P);
  P->nstrips = (p->nx + OWN - 1) / OWN;
  P->seg_rows = p->tile_rows > 0 ? p->tile_rows : default_tile_rows(*p, P->nstrips);
  if (p->flags & DUGKS_FLAG_MASS_FIX)   // whole mass groups per segment
    P->seg_rows = (P->seg_rows + MASS_GROUP - 1) / MASS_GROUP * MASS_GROUP;
  if (P->seg_rows > p->ny) P->seg_rows = p->ny;
  P->nsegs = (p->ny + P->seg_rows - 1) / P->seg_rows;
  *out = P;
  return DUGKS_OK;
}

void dugks_plan_destroy(dugks_plan* plan) {
  if (!plan) return;
  if (plan->head) (void)hipHostFree(plan->head);
  delete plan;
}

size_t dugks_state_bytes(const dugks_plan* plan) { return plan ? plan->L.total : 0; }

int dugks_init(const dugks_plan* plan, void* state, const double* phi0_dev,
               const double* uv_dev, void* stream) {
  if (!plan || !state || !phi0_dev || !aligned(state)) return DUGKS_EINVAL;
  if (plan->p.vel_kind == DUGKS_VEL_ARRAYS && !uv_dev) return DUGKS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return plan->p.precision == DUGKS_F64 ? do_init<double>(plan, state, phi0_dev, uv_dev, s)
                                        : do_init<float>(plan, state, phi0_dev, uv_dev, s);
}

int dugks_step(const dugks_plan* plan, void* state, int64_t step, int64_t nsteps,
               void* stream) {
  if (!plan || !state || !aligned(state) || step < 0 || nsteps < 0) return DUGKS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int64_t k = 0; k < nsteps; k++) {
    int rc = plan->p.precision == DUGKS_F64 ? launch_step<double>(plan, state, step + k, s)
                                            : launch_step<float>(plan, state, step + k, s);
    if (rc) return rc;
  }
  return DUGKS_OK;
}

int dugks_tune(const dugks_params* params, void* state, int64_t step, int32_t reps,
               int32_t* rows_out, void* stream) {
  if (!params || !state || !rows_out || !aligned(state) || step < 0 || reps < 1 || reps > 1000)
    return DUGKS_EINVAL;
  const int rc0 = validate(params);
  if (rc0) return rc0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // candidates: the default height, then 16..256 rows in steps of MASS_GROUP
  // (as the plans round them: duplicates dropped)
  std::vector<dugks_plan*> plans;
  int rc = DUGKS_OK;
  for (int c = 0; c <= std::min(256, params->ny) && !rc; c = (c == 0 ? 16 : c + MASS_GROUP)) {
    dugks_params q = *params;
    q.tile_rows = c;
    dugks_plan* P = nullptr;
    if ((rc = dugks_plan_create(&q, &P))) break;
    bool dup = false;
    for (dugks_plan* o : plans) dup = dup || o->seg_rows == P->seg_rows;
    if (dup)
      dugks_plan_destroy(P);
    else
      plans.push_back(P);
  }
  auto launch = [&](const dugks_plan* P) {
    return P->p.precision == DUGKS_F64 ? launch_step<double>(P, state, step, s, false)
                                       : launch_step<float>(P, state, step, s, false);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = DUGKS_EDEVICE;
  // the clocks ramp up over the first launches after idle: warm up first, then
  // time every candidate twice (forward, then backward) and keep its best
  for (int k = 0; k < 20 && !rc; k++) rc = launch(plans[0]);
  std::vector<float> best(plans.size(), 0.0f);
  for (int pass = 0; pass < 2 && !rc; pass++) {
    for (size_t j = 0; j < plans.size() && !rc; j++) {
      const size_t i = pass == 0 ? j : plans.size() - 1 - j;
      rc = launch(plans[i]);   // one untimed launch at this shape
      if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = DUGKS_EDEVICE;
      for (int k = 0; k < reps && !rc; k++) rc = launch(plans[i]);
      if (!rc && hipEventRecord(e1, s) != hipSuccess) rc = DUGKS_EDEVICE;
      float ms = 0.0f;
      if (!rc && (hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = DUGKS_EDEVICE;
      if (!rc && (pass == 0 || ms < best[i])) best[i] = ms;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (!rc) {
    size_t b = 0;
    for (size_t i = 1; i < plans.size(); i++)
      if (best[i] < best[b]) b = i;
    *rows_out = plans[b]->seg_rows;
  }
  for (dugks_plan* P : plans) dugks_plan_destroy(P);
  return rc;
}

int dugks_phi(const dugks_plan* plan, const void* state, int64_t step, void* phi_out_dev,
              void* stream) {
  if (!plan || !state || !phi_out_dev || !aligned(state) || step < 0) return DUGKS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return plan->p.precision == DUGKS_F64 ? do_phi<double>(plan, state, step, phi_out_dev, s)
                                        : do_phi<float>(plan, state, step, phi_out_dev, s);
}

int dugks_distributions(const dugks_plan* plan, const void* state, int64_t step,
                        void* out_dev, void* stream) {
  if (!plan || !state || !out_dev || !aligned(state) || step < 0) return DUGKS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return plan->p.precision == DUGKS_F64 ? do_export<double>(plan, state, step, out_dev, s)
                                        : do_export<float>(plan, state, step, out_dev, s);
}

int dugks_history(const dugks_plan* plan, const void* state, int64_t step, void* out_dev,
                  void* stream) {
  if (!plan || !state || !out_dev || !aligned(state) || step < 0) return DUGKS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return plan->p.precision == DUGKS_F64 ? do_history<double>(plan, state, step, out_dev, s)
                                        : do_history<float>(plan, state, step, out_dev, s);
}

int dugks_state_status(const dugks_plan* plan, const void* state, int32_t* status_out,
                 void* stream) {
  if (!plan || !state || !status_out || !aligned(state)) return DUGKS_EINVAL;
  const StateHeader* hd = at<StateHeader>(state, 0);
  return hip_status(hipMemcpyAsync(status_out, &hd->status, sizeof(int32_t), hipMemcpyDefault,
                                   static_cast<hipStream_t>(stream)));
}

int dugks_mass(const dugks_plan* plan, void* state, int64_t step, double* mass_out_dev,
               void* stream) {
  if (!plan || !state || !mass_out_dev || !aligned(state) || step < 0) return DUGKS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return plan->p.precision == DUGKS_F64 ? do_mass<double>(plan, state, step, mass_out_dev, s)
                                        : do_mass<float>(plan, state, step, mass_out_dev, s);
}

int dugks_mass_correct(const dugks_plan* plan, void* state, int64_t step, void* stream) {
  if (!plan || !state || !aligned(state) || step < 0) return DUGKS_EINVAL;
  if (plan->p.precision == DUGKS_F64 || (plan->p.flags & DUGKS_FLAG_MASS_FIX)) return DUGKS_OK;
  return do_correct<float>(plan, state, step, static_cast<hipStream_t>(stream));
}

int dugks_mass0(const dugks_plan* plan, const void* state, double* out_dev, void* stream) {
  if (!plan || !state || !out_dev || !aligned(state)) return DUGKS_EINVAL;
  const StateHeader* hd = at<StateHeader>(state, 0);
  return hip_status(hipMemcpyAsync(out_dev, &hd->mass0, sizeof(double),
                                   hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
}

const char* dugks_strerror(int status) {
  switch (status) {
    case DUGKS_OK: return "ok";
    case DUGKS_EINVAL: return "invalid argument";
    case DUGKS_ENOMEM: return "out of host memory";
    case DUGKS_EDEVICE: return "HIP launch or runtime call failed";
    case DUGKS_ENUMERIC: return "non-finite total mass";
    case DUGKS_EUNSUPPORTED: return "not supported by this library";
    default: return "unknown status";
  }
}

const char* dugks_version(void) { return "dugks-gfx950 0.1"; }

}  // extern "C"
