// dugks_kernels.h -- device kernels of one D2Q9 DUGKS (T2) step for the
// conservative Allen-Cahn equation (arXiv 2007.07760, Sec. II).
//
// The fused step kernel: one wavefront owns a strip of OWN = 58 columns (its 64
// lanes carry 3 halo columns each side) and marches up a segment of rows.  Per
// row it
//   - loads the 9 f~ planes and the phi history of row r+1 (coalesced, x fastest),
//   - forms phi (Eq. 30) into an LDS ring,
//   - at row r: the isotropic normal, theta (Eqs. 2, 4), d(phi u)/dt, and from
//     Eq. (14) feq and S collapsed into fbar+ (Eq. 23, LDS ring of 4-5 rows) and
//     f~+ (Eq. 9, registers),
//   - at row k = r-2: the face values fbar(x_b, t+h) of the east and north face
//     of each cell (Eqs. 24-26, each a fixed stencil of <= 20 taps with
//     coefficients built on the host), phi_b (Eq. 28), feq_b, S_b and f_b
//     (Eq. 27), the meso-flux (Eq. 21) and the update f~^{n+1} = f~+ + dt L,
// and writes f~^{n+1} and phi^n of its own cells.  Neighbour columns come from
// LDS, the own column's pipeline lives in registers; the loop is unrolled by 3
// so the register ring rotates without moves.
#pragma once

#include "dugks_common.h"

namespace dugks {

// Scalars of one grid.  The buffers go to the kernel as separate __restrict__
// parameters: only there does the compiler take them as non-aliasing, which
// lets the uniform coefficient and table reads use the scalar cache.
template <typename T>
struct StepArgs {
  int64_t pitch, plane;
  int nx, ny;
  int seg_rows, nstrips, nsegs, nlogical;
  T cA, cB;       // f~+   = cA f~ + cB (feq + tau S)
  T cA2, cB2;     // fbar+ = cA2 f~ + cB2 (feq + tau S)
  T dalpha;       // dt * 2tau/(2tau+h)
  T dt, beta, gamma, tau, kth;   // kth = 4/W (0: theta off)
  double period;  // time modulation cos(pi t / period); 0 = steady
  double dtd, hd; // dt, h in FP64 for the time factors
  int jzero;      // 1: d(phi u)/dt = 0 on every step
};

template <typename T>
struct RowRegs {
  T f[9];
  T hp;
};
template <typename T>
struct TfpRegs {
  T v[9];
};

__device__ __forceinline__ int wrapi(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

template <typename T>
struct StepBufs {
  const T* __restrict__ src;     // f~^n, 9 planes
  T* __restrict__ dst;           // f~^{n+1}, 9 planes
  const T* __restrict__ ph_src;  // phi^{n-1}
  T* __restrict__ ph_dst;        // phi^n
  const T* __restrict__ cf;      // [2][9][NTAP] face stencils
  const T* __restrict__ tabx;    // UX[2nx+2], VX[2nx+2]
  const T* __restrict__ taby;    // UY[2ny+2], VY[2ny+2]
};

template <typename T, int R>
struct Marcher {
  static constexpr int RB = (R == DUGKS_CENTRAL4) ? 5 : 4;

  const StepArgs<T>& a;
  const T* __restrict__ src;
  T* __restrict__ dst;
  const T* __restrict__ ph_src;
  T* __restrict__ ph_dst;
  const T* __restrict__ cf;
  const T* __restrict__ tabx;
  const T* __restrict__ taby;
  T (*bfp)[9][LROW];   // [RB][9][LROW]
  T (*phl)[LROW];      // [4][LROW]
  T (*svl)[2][LROW];   // [3][2][LROW]
  T (*fel)[LROW];      // [6][LROW]
  int lane, col;
  bool owned;
  int y0, y1, base;
  T UXc, VXc, UXe, VXe;
  T gN, gP, gH, jscale;

  __device__ __forceinline__ int slotB(int row) const { return (row - base) % RB; }
  __device__ __forceinline__ int slot4(int row) const { return (row - base) & 3; }
  __device__ __forceinline__ int slot3(int row) const { return (row - base) % 3; }

  __device__ __forceinline__ void load_row(RowRegs<T>& d, int row) const {
    int rr = wrapi(row, a.ny);
    const T* p = src + (int64_t)rr * a.pitch + col;
#pragma unroll
    for (int i = 0; i < 9; i++) d.f[i] = p[(int64_t)i * a.plane];
    d.hp = ph_src[(int64_t)rr * a.pitch + col];
  }

  // phi = sum_i f~_i (Eq. 30), same summation order as a plain loop over i
  __device__ __forceinline__ void phi_stage(const RowRegs<T>& d, int row) const {
    T s = d.f[0];
#pragma unroll
    for (int i = 1; i < 9; i++) s += d.f[i];
    phl[slot4(row)][LPAD + lane] = s;
  }

  // cell-centred terms of row r: normal, theta, d(phi u)/dt, S, feq -> fbar+
  // into the LDS ring and f~+ into registers
  __device__ __forceinline__ void cell_stage(const RowRegs<T>& d, int r,
                                             TfpRegs<T>& tp) const {
    const int L = LPAD + lane;
    const T* pm = phl[slot4(r - 1)];
    const T* p0 = phl[slot4(r)];
    const T* pp = phl[slot4(r + 1)];
    const T pC = p0[L];
    const T pE = p0[L + 1], pW = p0[L - 1], pN = pp[L], pS = pm[L];
    const T pNE = pp[L + 1], pNW = pp[L - 1], pSE = pm[L + 1], pSW = pm[L - 1];
    // isotropic gradient: (1/RT) sum_k w_k e_k phi_k
    const T third = T(1) / T(3), twelfth = T(1) / T(12);
    T gx = (pE - pW) * third + ((pNE - pNW) + (pSE - pSW)) * twelfth;
    T gy = (pN - pS) * third + ((pNE - pSE) + (pNW - pSW)) * twelfth;
    T gm = sqrt(gx * gx + gy * gy);
    T den = gm > T(1e-12) ? gm : T(1e-12);
    T th = a.kth * pC * (T(1) - pC) / den;     // theta / |grad phi|
    int rr = wrapi(r, a.ny);
    T UYr = taby[2 * rr + 1];
    T VYr = taby[(2 * a.ny + 2) + 2 * rr + 1];
    T Uc = UXc * UYr, Vc = VXc * VYr;          // spatial part of u at the cell
    T dj = (gN * pC - gP * d.hp) * jscale;     // d(phi g)/dt
    T sx = th * gx + T(3) * (Uc * dj);         // s = theta n + J / RT
    T sy = th * gy + T(3) * (Vc * dj);
    svl[slot3(r)][0][L] = sx;
    svl[slot3(r)][1][L] = sy;
    // feq + tau S = w_i (phi + e_i . m),  m = phi u / RT + tau s
    T uc = gN * Uc, vc = gN * Vc;
    T mx = T(3) * pC * uc + a.tau * sx;
    T my = T(3) * pC * vc + a.tau * sy;
    T* bf = &bfp[slotB(r)][0][0];
#pragma unroll
    for (int i = 0; i < 9; i++) {
      T em = pC;
      if (ex(i) > 0) em += mx;
      if (ex(i) < 0) em -= mx;
      if (ey(i) > 0) em += my;
      if (ey(i) < 0) em -= my;
      T X = T(wq(i)) * em;
      bf[i * LROW + L] = a.cA2 * d.f[i] + a.cB2 * X;
      tp.v[i] = a.cA * d.f[i] + a.cB * X;
    }
  }

  // reconstruction of one face value from the fbar+ ring
  template <int O>
  __device__ __forceinline__ T recon(int i, int k) const {
    const int L = LPAD + lane;
    const T* c = cf + (O * 9 + i) * NTAP;
    T v = T(0);
#pragma unroll
    for (int t = 0; t < NTAP; t++) {
      if (tap_used(R, O, i, t)) {
        const T f = bfp[slotB(k + tap_dy(O, t))][i][L + tap_dx(O, t)];
        v = fma(c[t], f, v);
      }
    }
    return v;
  }

  // faces of row k and the update of its cells
  __device__ __forceinline__ void face_stage(int k, const TfpRegs<T>& tp, T (&fS)[9],
                                             bool do_update) const {
    const int L = LPAD + lane;
    T bN[9], bE[9];
    T phN = T(0), phE = T(0);
#pragma unroll
    for (int i = 0; i < 9; i++) {
      bN[i] = recon<1>(i, k);
      phN += bN[i];
      if (do_update) {
        bE[i] = recon<0>(i, k);
        phE += bE[i];
      }
    }
    const int kk = wrapi(k, a.ny);
    const T* UY = taby;
    const T* VY = taby + (2 * a.ny + 2);
    // north face (x + 1/2, y + 1): S_b = mean of the two cells (own column)
    {
      T sx = T(0.5) * (svl[slot3(k)][0][L] + svl[slot3(k + 1)][0][L]);
      T sy = T(0.5) * (svl[slot3(k)][1][L] + svl[slot3(k + 1)][1][L]);
      T ub = gH * (UXc * UY[2 * kk + 2]);
      T vb = gH * (VXc * VY[2 * kk + 2]);
      T P = a.beta * phN;
      T Qx = T(3) * P * ub + a.gamma * sx;
      T Qy = T(3) * P * vb + a.gamma * sy;
#pragma unroll
      for (int i = 0; i < 9; i++) {
        if (ey(i) == 0) continue;
        T em = P;
        if (ex(i) > 0) em += Qx;
        if (ex(i) < 0) em -= Qx;
        if (ey(i) > 0) em += Qy;
        if (ey(i) < 0) em -= Qy;
        T fN = a.dalpha * bN[i] + (a.dt * T(wq(i))) * em;
        if (do_update) {
          T d = fN - fS[i];
          bN[i] = ey(i) > 0 ? d : -d;   // e_iy (fN - fS), reuse bN
        }
        fS[i] = fN;
      }
    }
    if (!do_update) return;
    // east face (x + 1, y + 1/2): S_b = mean of own and east cell
    T fE[9];
    {
      T sx = T(0.5) * (svl[slot3(k)][0][L] + svl[slot3(k)][0][L + 1]);
      T sy = T(0.5) * (svl[slot3(k)][1][L] + svl[slot3(k)][1][L + 1]);
      T ub = gH * (UXe * UY[2 * kk + 1]);
      T vb = gH * (VXe * VY[2 * kk + 1]);
      T P = a.beta * phE;
      T Qx = T(3) * P * ub + a.gamma * sx;
      T Qy = T(3) * P * vb + a.gamma * sy;
      int q = 0;
#pragma unroll
      for (int i = 0; i < 9; i++) {
        if (ex(i) == 0) continue;
        T em = P;
        if (ex(i) > 0) em += Qx;
        if (ex(i) < 0) em -= Qx;
        if (ey(i) > 0) em += Qy;
        if (ey(i) < 0) em -= Qy;
        fE[i] = a.dalpha * bE[i] + (a.dt * T(wq(i))) * em;
        fel[q][L] = fE[i];
        q++;
      }
    }
    __syncthreads();
    // west face of this cell = east face of the lane to the left; update
    T out[9];
    {
      int q = 0;
#pragma unroll
      for (int i = 0; i < 9; i++) {
        T flux = T(0);
        if (ex(i) != 0) {
          T d = fE[i] - fel[q][L - 1];
          flux = ex(i) > 0 ? d : -d;
          q++;
        }
        if (ey(i) != 0) flux += bN[i];
        out[i] = tp.v[i] - flux;
      }
    }
    if (owned) {
      const int64_t o = (int64_t)kk * a.pitch + col;
#pragma unroll
      for (int i = 0; i < 9; i++) dst[(int64_t)i * a.plane + o] = out[i];
      ph_dst[o] = phl[slot4(k)][L];
    }
  }

  // one row of the march: load r+2, phi of r+1, cell terms of r, faces of r-2
  __device__ __forceinline__ void body(int r, RowRegs<T>& B, RowRegs<T>& C,
                                       RowRegs<T>& D, TfpRegs<T>& Pr,
                                       TfpRegs<T>& Pk, T (&fS)[9]) const {
    if (r > y1 + 1) return;
    if (r + 2 <= y1 + 2) load_row(D, r + 2);
    phi_stage(C, r + 1);
    __syncthreads();
    cell_stage(B, r, Pr);
    __syncthreads();
    const int k = r - 2;
    if (k >= y0 - 1) face_stage(k, Pk, fS, k >= y0);
  }

  __device__ void run() {
    RowRegs<T> B, C, D;
    TfpRegs<T> P0, P1, P2;
    T fS[9];
#pragma unroll
    for (int i = 0; i < 9; i++) fS[i] = T(0);
    load_row(C, y0 - 3);
    phi_stage(C, y0 - 3);
    load_row(B, y0 - 2);
    phi_stage(B, y0 - 2);
    load_row(C, y0 - 1);
    // r = y0-2 + 3j + {0,1,2}; tf~+ of row r sits in P[(r - y0 + 2) % 3] and
    // that of row r-2 in P[(r - y0 + 3) % 3]
    for (int r = y0 - 2; r <= y1 + 1; r += 3) {
      body(r, B, C, D, P0, P1, fS);
      body(r + 1, C, D, B, P1, P2, fS);
      body(r + 2, D, B, C, P2, P0, fS);
    }
  }
};

template <typename T, int R>
__global__ __launch_bounds__(LANES) void step_kernel(
    StepArgs<T> a, int64_t n, const T* __restrict__ src, T* __restrict__ dst,
    const T* __restrict__ ph_src, T* __restrict__ ph_dst, const T* __restrict__ cf,
    const T* __restrict__ tabx, const T* __restrict__ taby) {
  constexpr int RB = Marcher<T, R>::RB;
  __shared__ T s_bfp[RB][9][LROW];
  __shared__ T s_phi[4][LROW];
  __shared__ T s_sv[3][2][LROW];
  __shared__ T s_fe[6][LROW];

  // XCD-aware order: consecutive blocks go round-robin to the 8 XCDs, so give
  // each XCD a contiguous band of tiles (shared halos stay in one L2)
  const int per = (a.nlogical + 7) >> 3;
  const int logical = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (logical >= a.nlogical) return;
  const int strip = logical % a.nstrips;
  const int seg = logical / a.nstrips;

  const int lane = threadIdx.x;
  // zero the LDS pads once (never read by owned results, kept finite)
  for (int j = lane; j < RB * 9 * LROW; j += LANES) (&s_bfp[0][0][0])[j] = T(0);
  for (int j = lane; j < 4 * LROW; j += LANES) (&s_phi[0][0])[j] = T(0);
  for (int j = lane; j < 3 * 2 * LROW; j += LANES) (&s_sv[0][0][0])[j] = T(0);
  for (int j = lane; j < 6 * LROW; j += LANES) (&s_fe[0][0])[j] = T(0);
  __syncthreads();

  Marcher<T, R> m{a, src, dst, ph_src, ph_dst, cf, tabx, taby, s_bfp, s_phi, s_sv, s_fe};
  const int x0 = strip * OWN;
  m.lane = lane;
  int c0 = (x0 - HALO + lane) % a.nx;
  m.col = c0 < 0 ? c0 + a.nx : c0;
  const int nown = min(OWN, a.nx - x0);
  m.owned = lane >= HALO && lane < HALO + nown;
  m.y0 = seg * a.seg_rows;
  m.y1 = min(m.y0 + a.seg_rows, a.ny);
  m.base = m.y0 - 3;
  const int ce = m.col + 1;  // east face of the column (x + 1), unwrapped
  m.UXc = tabx[2 * m.col + 1];
  m.VXc = tabx[(2 * a.nx + 2) + 2 * m.col + 1];
  m.UXe = tabx[2 * ce];
  m.VXe = tabx[(2 * a.nx + 2) + 2 * ce];
  // time factors of the velocity at t_n, t_{n-1} (cells) and t_n + h (faces)
  const double tn = (double)n * a.dtd;
  double gn = 1.0, gp = 1.0, gh = 1.0;
  if (a.period > 0.0) {
    gn = cos(M_PI * tn / a.period);
    gp = cos(M_PI * (tn - a.dtd) / a.period);
    gh = cos(M_PI * (tn + a.hd) / a.period);
  }
  m.gN = T(gn);
  m.gP = T(gp);
  m.gH = T(gh);
  m.jscale = (n == 0 || a.jzero) ? T(0) : T(1) / a.dt;
  m.run();
}

// ------------------------------------------------------------------ init
template <typename T>
struct InitArgs {
  const double* __restrict__ phi0;  // [ny][nx] dense
  T* __restrict__ tf;               // 9 planes
  T* __restrict__ ph;               // phi history plane
  const T* __restrict__ tabx;
  const T* __restrict__ taby;
  int64_t pitch, plane;
  int nx, ny;
  double dt, kth;
};

// f~^0 = feq(phi0, u(x,0)) - (dt/2) S^0 with d(phi u)/dt = 0
template <typename T>
__global__ __launch_bounds__(256) void init_kernel(InitArgs<T> a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= a.nx || y >= a.ny) return;
  auto P = [&](int dx, int dy) {
    return a.phi0[(int64_t)wrapi(y + dy, a.ny) * a.nx + wrapi(x + dx, a.nx)];
  };
  const double pC = P(0, 0);
  const double gx = (P(1, 0) - P(-1, 0)) / 3.0 +
                    ((P(1, 1) - P(-1, 1)) + (P(1, -1) - P(-1, -1))) / 12.0;
  const double gy = (P(0, 1) - P(0, -1)) / 3.0 +
                    ((P(1, 1) - P(1, -1)) + (P(-1, 1) - P(-1, -1))) / 12.0;
  const double gm = sqrt(gx * gx + gy * gy);
  const double den = gm > 1e-12 ? gm : 1e-12;
  const double th = a.kth * pC * (1.0 - pC);
  const double nvx = gx / den, nvy = gy / den;
  const double u = (double)a.tabx[2 * x + 1] * (double)a.taby[2 * y + 1];
  const double v = (double)a.tabx[(2 * a.nx + 2) + 2 * x + 1] *
                   (double)a.taby[(2 * a.ny + 2) + 2 * y + 1];
  const int64_t o = (int64_t)y * a.pitch + x;
#pragma unroll
  for (int i = 0; i < 9; i++) {
    const double eu = ex(i) * u + ey(i) * v;
    const double en = ex(i) * nvx + ey(i) * nvy;
    const double feq = wq(i) * pC * (1.0 + 3.0 * eu);
    const double src = wq(i) * th * en;
    a.tf[(int64_t)i * a.plane + o] = T(feq - 0.5 * a.dt * src);
  }
  a.ph[o] = T(pC);
}

// ------------------------------------------------------------------ phi
template <typename T>
__global__ __launch_bounds__(256) void phi_kernel(const T* __restrict__ tf,
                                                  int64_t pitch, int64_t plane,
                                                  int nx, int ny,
                                                  T* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= nx || y >= ny) return;
  const int64_t o = (int64_t)y * pitch + x;
  T s = tf[o];
#pragma unroll
  for (int i = 1; i < 9; i++) s += tf[(int64_t)i * plane + o];
  out[(int64_t)y * nx + x] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void export_kernel(const T* __restrict__ tf, int64_t pitch,
                                                     int64_t plane, int nx, int ny,
                                                     T* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  const int i = blockIdx.z;
  if (x >= nx || y >= ny) return;
  out[((int64_t)i * ny + y) * nx + x] = tf[(int64_t)i * plane + (int64_t)y * pitch + x];
}

// ------------------------------------------------------------------ mass
// Neumaier pair (sum, compensation)
__device__ __forceinline__ void neu_add(double& s, double& c, double v) {
  double t = s + v;
  if (fabs(s) >= fabs(v))
    c += (s - t) + v;
  else
    c += (v - t) + s;
  s = t;
}

// block partials of sum(phi) over a fixed cell partition: partial b covers the
// cells b, b + MASS_BLOCKS*MASS_THREADS, ... of thread order; every reduction
// order is fixed, so the result is bitwise reproducible.
template <typename T, int NPL>
__global__ __launch_bounds__(MASS_THREADS) void mass_partial_kernel(
    const T* __restrict__ tf, int64_t pitch, int64_t plane, int nx, int ny,
    double* __restrict__ part) {
  __shared__ double ss[MASS_THREADS], sc[MASS_THREADS];
  const int64_t N = (int64_t)nx * ny;
  double s = 0.0, c = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * MASS_THREADS + threadIdx.x; j < N;
       j += (int64_t)MASS_BLOCKS * MASS_THREADS) {
    const int y = (int)(j / nx), x = (int)(j % nx);
    const int64_t o = (int64_t)y * pitch + x;
    double v = (double)tf[o];
#pragma unroll
    for (int i = 1; i < NPL; i++) v += (double)tf[(int64_t)i * plane + o];
    neu_add(s, c, v);
  }
  ss[threadIdx.x] = s;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int w = MASS_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      double a = ss[threadIdx.x], ac = sc[threadIdx.x] + sc[threadIdx.x + w];
      neu_add(a, ac, ss[threadIdx.x + w]);
      ss[threadIdx.x] = a;
      sc[threadIdx.x] = ac;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ss[0];
    part[2 * blockIdx.x + 1] = sc[0];
  }
}

__global__ __launch_bounds__(64) void mass_final_kernel(const double* __restrict__ part,
                                                        double* __restrict__ out,
                                                        double* __restrict__ out2) {
  if (threadIdx.x != 0) return;
  double s = 0.0, c = 0.0;
  for (int b = 0; b < MASS_BLOCKS; b++) {
    c += part[2 * b + 1];
    neu_add(s, c, part[2 * b]);
  }
  const double m = s + c;
  *out = m;
  if (out2) *out2 = m;
}

// f~_i += w_i (M0 - M) / (nx ny)
template <typename T>
__global__ __launch_bounds__(256) void mass_correct_kernel(
    T* __restrict__ tf, int64_t pitch, int64_t plane, int nx, int ny,
    const StateHeader* __restrict__ hdr) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= nx || y >= ny) return;
  const double delta = (hdr->mass0 - hdr->mass_now) / ((double)nx * (double)ny);
  const int64_t o = (int64_t)y * pitch + x;
#pragma unroll
  for (int i = 0; i < 9; i++) {
    T& f = tf[(int64_t)i * plane + o];
    f = T((double)f + wq(i) * delta);
  }
}

}  // namespace dugks
