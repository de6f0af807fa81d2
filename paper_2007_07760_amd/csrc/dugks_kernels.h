// dugks_kernels.h -- device kernels of one D2Q9 DUGKS step for the
// conservative Allen-Cahn equation (arXiv 2007.07760, Sec. II): the T2 step
// and the two stages of the T3S3 step.
//
// The fused step kernel: one wavefront owns a strip of OWN = 58 columns (its 64
// lanes carry 3 halo columns each side) and marches up a segment of rows.  At
// row r it
//   - sums phi (Eq. 30) of row r+1 (loaded one row earlier) and keeps phi and
//     its horizontal differences in registers,
//   - forms, at the cells of row r, the isotropic normal, theta (Eqs. 2, 4),
//     d(phi u)/dt and from Eq. (14) feq and S, collapsed into X = feq + tau S
//     and fbar+ (Eq. 23) -> an LDS ring of 4 rows (5 for central-4),
//   - issues the loads of row r+2 (the 9 f~ planes and the phi history,
//     coalesced, x fastest),
//   - at row k = r-2: the face values fbar(x_b, t+h) of the east and north face
//     of each cell (Eqs. 24-26, each a fixed stencil of <= 20 taps with
//     coefficients built on the host), phi_b (Eq. 28), feq_b, S_b and f_b
//     (Eq. 27), the meso-flux (Eq. 21) and the update f~^{n+1} = f~+ + dt L
//     with f~+ (Eq. 9) rebuilt from fbar+ and X,
// and writes f~^{n+1} and phi^n of its own cells.  Neighbour columns come from
// LDS or DPP lane shifts; the own column's pipeline lives in registers.  The
// first rows of a tile (no faces yet) are peeled off the loop, so that every
// row of the loop issues the same loads and stores and the waits for the loads
// never cover stores.
#pragma once

#include "dugks_common.h"

namespace dugks {

// Scalars of one grid.  The buffers go to the kernel as separate __restrict__
// parameters: only there does the compiler take them as non-aliasing, which
// lets the uniform coefficient and table reads use the scalar cache.
template <typename T>
struct StepArgs {
  int64_t CH;            // strip-chunk length (elements), see Tiling
  int nx, ny;
  int seg_rows, nstrips, nsegs, nlogical;
  int ileave, clen;      // tile order of step_kernel (see there)
  int ngroups;           // row groups of MASS_GROUP rows (mass partials)
  T cB2;                 // fbar+ = g + cB2 (feq + tau S - g), g the stage's input
  T kap;                 // output = base + kap (feq + tau S - fbar+) + wo1 dt L
  T wo1, wo2;            // weights of dt L in the outputs (see Stage)
  T pscale;              // beta / alpha (the stencil table carries dt*alpha)
  T gdt;                 // dt * gamma / 2 (face S is the mean of two cells)
  T dt, tau, kth;        // kth = 4/W (0: theta off)
  T jinv;                // 1 / (time between the two phi of d(phi u)/dt)
  double period;  // time modulation cos(pi t / period); 0 = steady
  double dtd, hd; // dt; the stage's half step (faces at base time + hd)
  double toff;    // base time of the stage: n dt + toff
  double troff;   // time of the earlier phi of d(phi u)/dt: n dt + troff
  int jzero;      // 1: d(phi u)/dt = 0 on every step
  int jfirst;     // 1: d(phi u)/dt = 0 on step 0 (no earlier phi yet)
};

// The launches of one time step.  T2: f~^n -> f~^{n+1} (Sec. II.B.1).  T3S3
// (Sec. II.B.2) runs two: stage A reads f^^n, builds fbar+ with the half step
// dt/6 (Eq. 31) and writes f~ at t_n + dt/3 (Eqs. 15, 33) and
// Q = f^n + (3/7) dt L(f*) (Eq. 32 and the first flux term of Eq. 16); stage B
// reads f~ at t_n + dt/3, builds fbar+ with the half step 5 dt/12 (Eq. 34) and
// writes f^^{n+1} = Q + (3/4) dt (Omega + S) + (4/7) dt L(f**) (Eqs. 16, 29).
enum Stage { STAGE_T2 = 0, STAGE_A = 1, STAGE_B = 2 };

template <typename T>
struct StepBufs {
  const T* __restrict__ src;     // f~^n and phi^{n-1} (strip chunks)
  T* __restrict__ dst;           // f~^{n+1} and phi^n
  const T* __restrict__ cf;      // compact face-stencil table [NCOMPACT]
  const T* __restrict__ tabx;    // UX[2nx+2], VX[2nx+2]
  const T* __restrict__ taby;    // UY[2ny+2], VY[2ny+2]
};

// Read-only tables that every lane of a wavefront reads at the same index
// (the face stencil, the y velocity factors): read through the constant
// address space, whose uniform loads go through the scalar cache into scalar
// registers whatever the compiler can prove about aliasing with the stores.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)p;
}

// copy of a struct read through the constant address space, word by word
template <typename S>
__device__ __forceinline__ S load_const(cptr<S> p) {
  static_assert(sizeof(S) % 4 == 0, "whole words");
  S v;
  const cptr<uint32_t> w = (cptr<uint32_t>)p;
  uint32_t* o = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(S) / 4); k++) o[k] = w[k];
  return v;
}

template <typename T>
struct RowRegs {
  T f[9];
  T hp;
  T g[9];     // wide patch, lanes 0 and 63: f~ of the column beyond the halo
};

__device__ __forceinline__ int wrapi(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Value of the lane to the right / left through the DPP wavefront shifts
// (wave_shl:1 moves lane i+1 into lane i, wave_shr:1 lane i-1).  The edge
// lane with no source (63 / 0) reads 0 (bound_ctrl), which makes each shift
// one instruction.  Nothing of lanes 0 and 63 reaches an owned cell: the owned
// lanes 3..60 read fbar+ of lanes 1..62 at most (central-4's tangential
// differences), whose values depend on phi of lanes 0..63 only, and every
// face a lane takes from a neighbour belongs to lanes 2..61.
template <int CTRL>
__device__ __forceinline__ float dpp_shift(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
template <typename T>
__device__ __forceinline__ T from_right(T v) { return dpp_shift<0x130>(v); }
template <typename T>
__device__ __forceinline__ T from_left(T v) { return dpp_shift<0x138>(v); }

// Stores (and stage B's loads of Q) through a buffer resource: a lane whose
// byte offset lies past the resource's size writes nothing / reads 0 (the
// hardware range check), so a row's stores are issued by every lane on every
// row and the wait counts of the loads that follow them are the same on every
// path.  aux 2 = nontemporal.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr unsigned OFF_NONE = 0x80000000u;
__device__ __forceinline__ rsrc_t make_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}
__device__ __forceinline__ void bstore(float v, rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, 2);
}
__device__ __forceinline__ float bload(rsrc_t r, unsigned off, float) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double bload(rsrc_t r, unsigned off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void bstore(double v, rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 2);
}

// Ordering point for LDS traffic inside the (single-wavefront) workgroup: a
// wavefront's LDS operations execute in program order, so only the compiler
// must not move them across this point; no wait for outstanding operations.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// X_i = (feq + tau S)_i = w_i (phi + e_i . m),  m = phi u / RT + tau s,
// per weight class and direction pair, the rest weight taking what the others
// leave so that sum_i X_i = phi with no systematic rounding bias
template <typename T>
__device__ __forceinline__ void collision_target(T pC, T mx, T my, T (&x)[9]) {
  const T w1 = T(1.0 / 9.0), w2 = T(1.0 / 36.0);
  const T P1 = w1 * pC, P2 = w2 * pC;
  const T X1 = w1 * mx, Y1 = w1 * my;
  const T X2 = w2 * mx, Y2 = w2 * my;
  const T dpp = X2 + Y2, dmp = Y2 - X2;
  x[0] = fma(T(-4), P1 + P2, pC);
  x[1] = P1 + X1; x[5] = P1 - X1;
  x[3] = P1 + Y1; x[7] = P1 - Y1;
  x[2] = P2 + dpp; x[6] = P2 - dpp;
  x[4] = P2 + dmp; x[8] = P2 - dmp;
}

// theta / max(|g|, NORMAL_EPS), the square root and the quotient rounded
// exactly (a hardware reciprocal square root in FP32 was ~1 % faster, but
// moved the FP32 field of the 64^2 translation by 5x more in L-inf)
template <typename T>
__device__ __forceinline__ T over_norm(T theta, T gx, T gy) {
  const T gm = sqrt(fma(gx, gx, gy * gy));
  return theta / (gm > T(NORMAL_EPS) ? gm : T(NORMAL_EPS));
}

// VARR: the velocity comes from caller-supplied cell arrays (steady; a face
// takes the mean of its two cells) instead of the separable tables.
template <typename T, int R, bool MFIX, int STAGE = STAGE_T2, bool VARR = false>
struct Marcher {
  // the wide (upwind-5) patch reaches 2 rows below and 3 above the face row
  // and 3 columns beyond a lane: a 6-row ring, faces 3 rows behind the cell
  // terms, and lanes 0 / 63 compute phi of the column beyond them as well
  // (so that fbar+ is right on every lane); the narrow patches: a 4-row ring
  // (5 for central-4), faces 2 rows behind
  static constexpr bool WIDE = wide(R);
  static constexpr int RB = WIDE ? 6 : ((R == DUGKS_CENTRAL4) ? 5 : 4);
  static constexpr int LAG = WIDE ? 3 : 2;
  static constexpr int LP = lpad(R);
  static constexpr int LR = lrow(R);
  // FP32: the relaxation increments X_i - g_i are made to sum to zero in the
  // rest direction (see cell_stage); FP64 rounds phi to 1e-16 and keeps the
  // plain increments, as the oracle writes them
  static constexpr bool ZSUM = sizeof(T) == 4;
  // the fused mass correction: the stored state's loads take the pending
  // correction (T2; T3S3 stage A, which reads f^^n), the state's writes give
  // the new mass partials (T2; stage B, which writes f^^{n+1})
  static constexpr bool FIX_LOAD = MFIX && STAGE != STAGE_B;
  static constexpr bool FIX_SUM = MFIX && STAGE != STAGE_A;

  const StepArgs<T>& a;
  const T* __restrict__ src;
  cptr<T> cf;
  const T* __restrict__ tabx;
  cptr<T> taby;
  const T* __restrict__ uv;   // VARR: u plane then v plane, [ny][nx]
  T (*bfp)[9][LR];     // [RB][9][LR] ring of fbar+ rows
  int lane, col;
  int ocol;                 // owned lanes: column within the strip
  // the strip's own chunk column of the output (rdst), of stage A's second
  // output Q (rdst2), of stage B's input Q (raux) and of the input itself
  // (rin: stage B reads phi^n there); the strip's mass partials
  rsrc_t rdst, rdst2, rpart, raux, rin;
  int64_t loff;             // chunk offset of the lane's column (strip, x % OWN)
  int64_t loffx;            // wide patch, lanes 0 / 63: that of the column beyond
  bool owned;
  int y0, y1, base;
  T UXc, VXc, UXe, VXe;
  T gN, gP, gH, jscale;
  // own-column pipeline (registers; index 0 is the face row k = r - LAG)
  T ph[LAG + 2];            // phi of rows r-LAG .. r+1
  T D0, D1, D2;             // phi(x+1) - phi(x-1) of rows r-1 .. r+1
  T A0, A1, A2;             // phi(x-1) + 4 phi(x) + phi(x+1) of rows r-1 .. r+1
  T sxp[LAG + 1], syp[LAG + 1];   // s = theta n + J/RT of rows r-LAG .. r
  T cp[LAG + 1], cx[LAG + 1], cy[LAG + 1];   // phi, m of rows r-LAG .. r
  T fS[9];                  // dt*alpha*fbar of the face below (north face of k-1)
  T PS, QSx, QSy;           // its collision part, see face_stage
  // mass correction (MFIX): the stored f~_i of the cells whose stored f~_0 is
  // below fitmax lack w_i delta, the correction set after the previous step;
  // cw0..2 = w_i delta per weight class.  Per row group the lane sums the phi
  // it writes (macc) and counts the cells it writes with f~_0 below
  // MASS_FIT_MAX (mcnt), the cells the next correction goes to; the group
  // totals go to part_row[2 g + 0 / 1].
  T cw0, cw1, cw2, fitmax;
  double macc, mcnt;
  double* part_row;


  // VARR: component c (0: u, 1: v) at the lane's cell of (wrapped) row rr;
  // rows are read again at the faces two rows later, from the caches
  __device__ __forceinline__ T uv_at(int c, int rr) const {
    return uv[((int64_t)c * a.ny + rr) * a.nx + col];
  }

  __device__ __forceinline__ int slotB(int row) const { return (row - base) % RB; }

  // the lane's column in row rr of the source; plane i sits i * OWN further,
  // which the loads take as an immediate offset
  __device__ __forceinline__ const T* row_src(int rr) const {
    return src + (int64_t)rr * a.CH + loff;
  }

  __device__ __forceinline__ void load_row(RowRegs<T>& d, int row) {
    const int rw = wrapi(row, a.ny);
    const T* p = row_src(rw);
#pragma unroll
    for (int i = 0; i < 9; i++) d.f[i] = p[i * OWN];
    if (FIX_LOAD) {
      // the pending w_i delta of the cell's weight class, or 0 (one select
      // per class instead of one per plane)
      const bool fit = d.f[0] < fitmax;
      const T c0 = fit ? cw0 : T(0), c1 = fit ? cw1 : T(0), c2 = fit ? cw2 : T(0);
#pragma unroll
      for (int i = 0; i < 9; i++) d.f[i] += i == 0 ? c0 : ((i & 1) ? c1 : c2);
    }
    d.hp = p[9 * OWN];
    if (WIDE && (lane == 0 || lane == LANES - 1)) {
      const T* q = src + (int64_t)rw * a.CH + loffx;
#pragma unroll
      for (int i = 0; i < 9; i++) d.g[i] = q[i * OWN];
      if (FIX_LOAD) {
        const bool fit = d.g[0] < fitmax;
        const T c0 = fit ? cw0 : T(0), c1 = fit ? cw1 : T(0), c2 = fit ? cw2 : T(0);
#pragma unroll
        for (int i = 0; i < 9; i++) d.g[i] += i == 0 ? c0 : ((i & 1) ? c1 : c2);
      }
    }
  }

  // phi = sum_i f~_i (Eq. 30, pairwise) of a new row and its horizontal
  // differences
  __device__ __forceinline__ void phi_push(const RowRegs<T>& d) {
    const T p = (((d.f[0] + d.f[1]) + (d.f[2] + d.f[3])) +
                 ((d.f[4] + d.f[5]) + (d.f[6] + d.f[7]))) + d.f[8];
    T pE = from_right(p), pW = from_left(p);
    if (WIDE) {
      // the edge lanes' outer neighbour: the column they loaded besides their own
      const T px = (((d.g[0] + d.g[1]) + (d.g[2] + d.g[3])) +
                    ((d.g[4] + d.g[5]) + (d.g[6] + d.g[7]))) + d.g[8];
      pW = lane == 0 ? px : pW;
      pE = lane == LANES - 1 ? px : pE;
    }
#pragma unroll
    for (int j = 0; j < LAG + 1; j++) ph[j] = ph[j + 1];
    ph[LAG + 1] = p;
    D0 = D1; D1 = D2; D2 = pE - pW;
    A0 = A1; A1 = A2; A2 = fma(T(4), p, pW + pE);
  }

  // cell-centred terms of row r: isotropic normal, theta (Eqs. 2, 4),
  // d(phi u)/dt, feq and S (Eq. 14) collapsed into fbar+ (Eq. 23) -> LDS ring
  __device__ __forceinline__ void cell_stage(const RowRegs<T>& d, int r) {
    const int L = LP + lane;
    const T twelfth = T(1) / T(12);
    // (1/RT) sum_k w_k e_k phi_k, column-summed
    const T gx = fma(T(4), D1, D0 + D2) * twelfth;
    const T gy = (A2 - A0) * twelfth;
    const T pC = ph[LAG];
    const T th = over_norm(a.kth * pC * (T(1) - pC), gx, gy);   // theta / |grad phi|
    const int rr = wrapi(r, a.ny);
    T Uc, Vc;                                      // spatial part of u
    if (VARR) {
      Uc = uv_at(0, rr);
      Vc = uv_at(1, rr);
    } else {
      Uc = UXc * taby[2 * rr + 1];
      Vc = VXc * taby[(2 * a.ny + 2) + 2 * rr + 1];
    }
    const T dj = fma(gN, pC, -(gP * d.hp)) * jscale;   // d(phi g)/dt
    const T sx = fma(th, gx, T(3) * (Uc * dj));        // s = theta n + J / RT
    const T sy = fma(th, gy, T(3) * (Vc * dj));
    const T mx = fma(a.tau, sx, T(3) * pC * (gN * Uc));
    const T my = fma(a.tau, sy, T(3) * pC * (gN * Vc));
#pragma unroll
    for (int j = 0; j < LAG; j++) {
      sxp[j] = sxp[j + 1]; syp[j] = syp[j + 1];
      cp[j] = cp[j + 1]; cx[j] = cx[j + 1]; cy[j] = cy[j + 1];
    }
    sxp[LAG] = sx; syp[LAG] = sy;
    cp[LAG] = pC; cx[LAG] = mx; cy[LAG] = my;
    T x[9];
    collision_target(pC, mx, my, x);
    // fbar+ in increment form, fbar+_i = f~_i + cB2 (X_i - f~_i): its moments
    // follow those of X.  The increments sum to zero (sum_i X_i = phi =
    // sum_i f~_i); in FP32 the rest direction enforces that in the arithmetic
    // of the others, so that the rounding of phi itself moves no mass (near
    // phi = 1 every cell rounds phi alike, and the plain increments made FP32
    // gain ~3e-9 of the total mass per step)
    T* bf = &bfp[slotB(r)][0][0];
    T dsum = T(0);
#pragma unroll
    for (int i = 1; i < 9; i++) {
      const T dx = x[i] - d.f[i];
      if (ZSUM) dsum += dx;
      bf[i * LR + L] = fma(a.cB2, dx, d.f[i]);
    }
    bf[L] = fma(a.cB2, ZSUM ? -dsum : x[0] - d.f[0], d.f[0]);
  }

  // one face value: fixed stencil over the fbar+ ring (Eqs. 24-26); the
  // coefficients come from the compact symmetric table (uniform, scalar
  // registers), the tap pattern is compile-time
  template <int O>
  __device__ __forceinline__ T recon(int i, int k) const {
    const int L = LP + lane;
    T v = T(0);
#pragma unroll
    for (int t = 0; t < ntap(R); t++) {
      if (tap_used(R, O, i, t)) {
        const T f = bfp[slotB(k + tap_dy(R, O, t))][i][L + tap_dx(R, O, t)];
        v = fma(cf[compact_index(R, O, i, t)], f, v);
      }
    }
    return v;
  }

  // Faces of row k and the update of its cells.  With phi_b = sum_i fbar_i,
  // Eq. (27) gives dt f_b,i = dt*alpha*fbar_i + dt w_i (P + e_i . Q),
  // P = beta phi_b, Q = 3 P u_b + gamma S_b/w-part, so the flux differences
  // split into a per-velocity part, accumulated as each fbar_i is formed, and
  // a collision part in the 3 numbers (P, Qx, Qy) of each face.
  template <bool upd>
  __device__ __forceinline__ void face_stage(int k) {
    const int L = LP + lane;
    const int kk = wrapi(k, a.ny);
    // stage B: Q of the row (Eq. 32 value) and phi^n, the history plane of
    // stage A's f~(t') (the input), read before the face work so that the
    // loads are in flight meanwhile; lanes outside the owned columns read
    // nothing (out-of-range offsets read 0)
    T qv[10];
    if (STAGE == STAGE_B && upd) {
      const unsigned oq = owned ? (unsigned)((kk * a.CH + ocol) * (int)sizeof(T)) : OFF_NONE;
#pragma unroll
      for (int i = 0; i < 9; i++) qv[i] = bload(raux, oq + i * (unsigned)(OWN * sizeof(T)), T(0));
      qv[9] = bload(rin, oq + 9 * (unsigned)(OWN * sizeof(T)), T(0));
    }
    T out[9];
    T phN = T(0), phE = T(0);
#pragma unroll
    for (int i = 0; i < 9; i++) {
      out[i] = T(0);
      const T pn = recon<1>(i, k);      // dt*alpha*fbar_i (scaled stencil)
      phN += pn;
      if (ey(i) != 0) {
        const T d = pn - fS[i];
        if (upd) out[i] = ey(i) > 0 ? -d : d;
        fS[i] = pn;
      }
      if (upd) {
        const T pe = recon<0>(i, k);
        phE += pe;
        if (ex(i) != 0) {
          const T d = pe - from_left(pe);
          out[i] = ex(i) > 0 ? out[i] - d : out[i] + d;
        }
      }
      // keep one velocity's taps live at a time; other wavefronts hide the
      // LDS latency
      __builtin_amdgcn_sched_barrier(0);
    }
    const cptr<T> UY = taby;
    const cptr<T> VY = taby + (2 * a.ny + 2);
    // north face (x + 1/2, y + 1): S_b = mean of the two cells; a velocity
    // array gives the mean of the two cells' velocities (steady)
    T ubN, vbN, uk = T(0), vk = T(0);
    if (VARR) {
      const int k1 = wrapi(k + 1, a.ny);
      uk = uv_at(0, kk);
      vk = uv_at(1, kk);
      ubN = T(0.5) * (uk + uv_at(0, k1));
      vbN = T(0.5) * (vk + uv_at(1, k1));
    } else {
      ubN = gH * (UXc * UY[2 * kk + 2]);
      vbN = gH * (VXc * VY[2 * kk + 2]);
    }
    // phN = dt*alpha*phi_b; P = beta phi_b, Q = 3 P u_b + gamma s_b, all
    // carried pre-multiplied by dt so that dt f_b,i = pn_i + w_i (P + e_i.Q)
    const T PN = a.pscale * phN;
    const T QNx = fma(T(3) * PN, ubN, a.gdt * (sxp[0] + sxp[1]));
    const T QNy = fma(T(3) * PN, vbN, a.gdt * (syp[0] + syp[1]));
    const T dP = PN - PS, dQx = QNx - QSx, dQy = QNy - QSy;
    PS = PN; QSx = QNx; QSy = QNy;
    if (!upd) return;
    {
      // i = 3, 7 (axis, w = 1/9) and 2, 4, 6, 8 (diagonal, w = 1/36)
      const T a1 = T(1.0 / 9.0) * dP, ay1 = T(1.0 / 9.0) * dQy;
      const T a2 = T(1.0 / 36.0) * dP, ax2 = T(1.0 / 36.0) * dQx, ay2 = T(1.0 / 36.0) * dQy;
      out[3] -= a1 + ay1;
      out[7] += a1 - ay1;
      out[2] -= (a2 + ax2) + ay2;
      out[4] -= (a2 - ax2) + ay2;
      out[6] += (a2 - ax2) - ay2;
      out[8] += (a2 + ax2) - ay2;
    }
    // east face (x + 1, y + 1/2): S_b = mean of own and east cell
    const T ubE = VARR ? T(0.5) * (uk + from_right(uk)) : gH * (UXe * UY[2 * kk + 1]);
    const T vbE = VARR ? T(0.5) * (vk + from_right(vk)) : gH * (VXe * VY[2 * kk + 1]);
    const T PE = a.pscale * phE;
    const T QEx = fma(T(3) * PE, ubE, a.gdt * (sxp[0] + from_right(sxp[0])));
    const T QEy = fma(T(3) * PE, vbE, a.gdt * (syp[0] + from_right(syp[0])));
    const T eP = PE - from_left(PE), eQx = QEx - from_left(QEx), eQy = QEy - from_left(QEy);
    {
      // i = 1, 5 (axis) and 2, 4, 6, 8 (diagonal)
      const T a1 = T(1.0 / 9.0) * eP, ax1 = T(1.0 / 9.0) * eQx;
      const T a2 = T(1.0 / 36.0) * eP, ax2 = T(1.0 / 36.0) * eQx, ay2 = T(1.0 / 36.0) * eQy;
      out[1] -= a1 + ax1;
      out[5] += a1 - ax1;
      out[2] -= (a2 + ax2) + ay2;
      out[8] -= (a2 + ax2) - ay2;
      out[6] += (a2 - ax2) - ay2;
      out[4] += (a2 - ax2) + ay2;
    }
    // f~+ and fbar+ both relax f~ towards X = feq + tau S (Eqs. 9, 23), so
    // f~+ = fbar+ + kap (X - fbar+): X of row k is rebuilt from its phi and m
    // (held since its cell stage) instead of reading f~ of the row again.
    // Then f~^{n+1} = f~+ + dt L (Eq. 21).  The T3S3 stages write their
    // outputs in the same form (see Stage).
    double cs = 0.0, cf0 = 0.0;
    {
      T x[9];
      collision_target(cp[0], cx[0], cy[0], x);
      // the new row is not read again by this launch: stream it past the
      // caches; lanes outside the owned columns store nothing
      const unsigned ob = owned ? (unsigned)((kk * a.CH + ocol) * (int)sizeof(T)) : OFF_NONE;
      constexpr unsigned PL = OWN * sizeof(T);
      // X - fbar+ (FP32: with a zero sum enforced in the rest direction, see
      // cell_stage), plane 0 last
      T dsum = T(0);
      if (STAGE == STAGE_T2) {
#pragma unroll
        for (int j = 0; j < 9; j++) {
          const int i = j < 8 ? j + 1 : 0;
          const T bp = bfp[slotB(k)][i][L];
          T dx = x[i] - bp;
          if (ZSUM) {
            if (i != 0) dsum += dx; else dx = -dsum;
          }
          const T tfp = fma(a.kap, dx, bp);
          const T v = tfp + out[i];
          bstore(v, rdst, ob + i * PL);
          if (FIX_SUM) {
            cs += (double)v;
            if (i == 0 && owned && v < T(MASS_FIT_MAX)) cf0 = 1.0;
          }
        }
        bstore(ph[0], rdst, ob + 9 * PL);
      } else if (STAGE == STAGE_A) {
        // f~(t') = f~+ + (1/3) dt L* and Q = f^n + (3/7) dt L*, with
        // f~+ = fbar+ + kap (X - fbar+) and f^n = fbar+ - kap (X - fbar+)
#pragma unroll
        for (int j = 0; j < 9; j++) {
          const int i = j < 8 ? j + 1 : 0;
          const T bp = bfp[slotB(k)][i][L];
          T d = x[i] - bp;
          if (ZSUM) {
            if (i != 0) dsum += d; else d = -dsum;
          }
          bstore(fma(a.wo1, out[i], fma(a.kap, d, bp)), rdst, ob + i * PL);
          bstore(fma(a.wo2, out[i], fma(-a.kap, d, bp)), rdst2, ob + i * PL);
        }
        bstore(ph[0], rdst, ob + 9 * PL);   // Q needs no history plane: stage B reads this one
      } else {
        // f^^{n+1} = Q + kap (X' - fbar+) + (4/7) dt L**, kap (X' - fbar+)
        // being (3/4) dt (Omega + S) at t'; phi^n goes on as the history
#pragma unroll
        for (int j = 0; j < 9; j++) {
          const int i = j < 8 ? j + 1 : 0;
          const T bp = bfp[slotB(k)][i][L];
          T dx = x[i] - bp;
          if (ZSUM) {
            if (i != 0) dsum += dx; else dx = -dsum;
          }
          const T v = fma(a.wo1, out[i], fma(a.kap, dx, qv[i]));
          bstore(v, rdst, ob + i * PL);
          if (FIX_SUM) {
            cs += (double)v;
            if (i == 0 && owned && v < T(MASS_FIT_MAX)) cf0 = 1.0;
          }
        }
        bstore(qv[9], rdst, ob + 9 * PL);
      }
    }
    if (FIX_SUM) {
      // phi^{n+1} of the row (owned lanes) into the group total; a group
      // never straddles two segments (segments are whole groups), so its sum
      // -- lanes in a fixed butterfly after rows in order -- does not depend
      // on the tiling
      macc += owned ? cs : 0.0;
      mcnt += cf0;
      const bool gend = (k & (MASS_GROUP - 1)) == MASS_GROUP - 1 || k == a.ny - 1;
      double v = 0.0, w = 0.0;
      if (gend) {
        v = macc;
        w = mcnt;
#pragma unroll
        for (int m = 1; m < LANES; m <<= 1) {
          v += __shfl_xor(v, m);
          w += __shfl_xor(w, m);
        }
        macc = 0.0;
        mcnt = 0.0;
      }
      // issued on every row; only lane 0 at the end of a group writes
      const unsigned po = (gend && lane == 0) ? (unsigned)(16 * (k / MASS_GROUP)) : OFF_NONE;
      bstore(v, rpart, po);
      bstore(w, rpart, po + 8);
    }
  }

  // row r of the march: phi of r+1, cell terms of r, load r+2 (the last rows
  // load row y1 + LAG again, so that every row issues the same loads), faces
  // of r-LAG (none for the first rows of the tile; the north faces only for
  // row y0 - 1, the south faces of row y0)
  template <int FACE>
  __device__ __forceinline__ void body(int r, RowRegs<T>& cur, RowRegs<T>& nxt) {
    phi_push(nxt);
    cell_stage(cur, r);
    load_row(cur, min(r + 2, y1 + LAG));
    wave_sync();
    if (FACE == 1) face_stage<false>(r - LAG);
    if (FACE == 2) face_stage<true>(r - LAG);
    wave_sync();
  }

  __device__ void run() {
    RowRegs<T> B, C;
    macc = mcnt = 0.0;
#pragma unroll
    for (int j = 0; j < LAG + 1; j++) sxp[j] = syp[j] = cp[j] = cx[j] = cy[j] = T(0);
#pragma unroll
    for (int j = 0; j < LAG + 2; j++) ph[j] = T(0);
    D0 = D1 = D2 = A0 = A1 = A2 = T(0);
    PS = QSx = QSy = T(0);
#pragma unroll
    for (int i = 0; i < 9; i++) fS[i] = T(0);
#pragma unroll
    for (int i = 0; i < 9; i++) B.g[i] = C.g[i] = T(0);
    // cell terms from row y0 - LAG (the lowest row the faces of row y0 - 1
    // reach), their phi from row y0 - LAG - 1
    load_row(C, y0 - LAG - 1);
    phi_push(C);
    load_row(B, y0 - LAG);
    phi_push(B);
    load_row(C, y0 - LAG + 1);
#pragma unroll
    for (int j = 0; j < 2 * LAG - 1; j++) {
      if (j & 1)
        body<0>(y0 - LAG + j, C, B);
      else
        body<0>(y0 - LAG + j, B, C);
    }
    body<1>(y0 + LAG - 1, C, B);
    // the first full row before the loop, so that the loop is entered, as it
    // is repeated, right after a full row's loads and stores: the waits for
    // the loads at its head then never include stores
    body<2>(y0 + LAG, B, C);
    int r = y0 + LAG + 1;
    for (; r + 1 <= y1 + LAG - 1; r += 2) {
      body<2>(r, C, B);
      body<2>(r + 1, B, C);
    }
    if (r <= y1 + LAG - 1) body<2>(r, C, B);
  }
};

// One tile: the strip `strip` of the grid, rows of segment `seg`, step n.
// pend = per-cell mass correction delta still to apply to the stored f~ of the
// cells whose stored f~_0 is below fitmax (MFIX).
template <typename T, int R, bool MFIX, int STAGE = STAGE_T2, bool VARR = false>
__device__ __forceinline__ void march_tile(const StepArgs<T>& a, int64_t n,
                                           const T* __restrict__ src, T* __restrict__ dst,
                                           T* __restrict__ dst2, const T* __restrict__ aux,
                                           const T* __restrict__ cf,
                                           const T* __restrict__ tabx,
                                           const T* __restrict__ taby,
                                           const T* __restrict__ uv,
                                           double* __restrict__ part, double pend,
                                           double fitmax, int strip,
                                           int seg, T (*s_bfp)[9][lrow(R)]) {
  using M = Marcher<T, R, MFIX, STAGE, VARR>;
  M m{a, src, as_const(cf), tabx, as_const(taby), uv, s_bfp};
  const int lane = threadIdx.x;
  const int x0 = strip * OWN;
  m.lane = lane;
  const int c0 = (x0 - HALO + lane) % a.nx;
  m.col = c0 < 0 ? c0 + a.nx : c0;
  {
    const int cs = m.col / OWN;
    m.loff = (int64_t)cs * a.ny * a.CH + (m.col - cs * OWN);
  }
  m.loffx = m.loff;
  if (M::WIDE && (lane == 0 || lane == LANES - 1)) {
    // the column beyond the lane, outwards (wrapped)
    int cx = lane == 0 ? m.col - 1 : m.col + 1;
    cx = cx < 0 ? cx + a.nx : (cx >= a.nx ? cx - a.nx : cx);
    const int cs = cx / OWN;
    m.loffx = (int64_t)cs * a.ny * a.CH + (cx - cs * OWN);
  }
  const int nown = min(OWN, a.nx - x0);
  m.owned = lane >= HALO && lane < HALO + nown;
  m.ocol = lane - HALO;
  {
    // the strip's own chunk column: ny rows of CH elements
    const int64_t c0 = (int64_t)strip * a.ny * a.CH;
    const unsigned nb = (unsigned)((int64_t)a.ny * a.CH * (int64_t)sizeof(T));
    m.rdst = make_rsrc(dst + c0, nb);
    m.rdst2 = make_rsrc((STAGE == STAGE_A ? dst2 : dst) + c0, nb);
    m.raux = make_rsrc((STAGE == STAGE_B ? aux : src) + c0, nb);   // used by stage B
    m.rin = make_rsrc(src + c0, nb);
  }
  m.y0 = seg * a.seg_rows;
  m.y1 = min(m.y0 + a.seg_rows, a.ny);
  m.base = m.y0 - M::LAG - 1;   // at or below every ring row the tile touches
  if (!VARR) {
    const int ce = m.col + 1;  // east face of the column (x + 1), unwrapped
    m.UXc = tabx[2 * m.col + 1];
    m.VXc = tabx[(2 * a.nx + 2) + 2 * m.col + 1];
    m.UXe = tabx[2 * ce];
    m.VXe = tabx[(2 * a.nx + 2) + 2 * ce];
  }
  // time factors of the velocity at the stage's base time and at the time of
  // the earlier phi (cells), and at base + its half step (faces)
  const double tn = (double)n * a.dtd;
  const double tb = tn + a.toff;
  double gn = 1.0, gp = 1.0, gh = 1.0;
  if (a.period > 0.0) {
    gn = cos(M_PI * tb / a.period);
    gp = cos(M_PI * (tn + a.troff) / a.period);
    gh = cos(M_PI * (tb + a.hd) / a.period);
  }
  m.gN = T(gn);
  m.gP = T(gp);
  m.gH = T(gh);
  m.jscale = ((n == 0 && a.jfirst) || a.jzero) ? T(0) : a.jinv;
  if (MFIX) {
    m.cw0 = T(wq(0) * pend);
    m.cw1 = T(wq(1) * pend);
    m.cw2 = T(wq(2) * pend);
    m.fitmax = T(fitmax);
    m.part_row = part + 2 * (int64_t)strip * a.ngroups;
    m.rpart = make_rsrc(m.part_row, (unsigned)(16 * a.ngroups));
  }
  m.run();
}

template <typename T, int R, bool MFIX, int STAGE, bool VARR>
__global__ __launch_bounds__(LANES, step_waves(sizeof(T), R, MFIX)) void
step_kernel(StepArgs<T> a, int64_t n, const T* __restrict__ src, T* __restrict__ dst,
            T* __restrict__ dst2, const T* __restrict__ aux, const T* __restrict__ cf,
            const T* __restrict__ tabx, const T* __restrict__ taby,
            const T* __restrict__ uv, double* __restrict__ part,
            const StateHeader* __restrict__ hdr) {
  constexpr int RB = Marcher<T, R, MFIX, STAGE, VARR>::RB;
  constexpr int LR = lrow(R);
  __shared__ T s_bfp[RB][9][LR];

  // XCD-aware order: consecutive blocks go round-robin to the 8 XCDs, so give
  // each XCD a contiguous band of tiles (shared halos stay in one L2).  With
  // ileave = C > 1 the band is whole segments, cut into C chunks of clen
  // segments whose tiles are taken in turn (segment i of every chunk, then
  // i + 1, ...): a tile then starts about when the one below it in its strip
  // ends, while the rows they share are still cached.  Blocks beyond the
  // band's segments exit at once.
  int strip, seg;
  if (a.ileave <= 1) {
    const int per = (a.nlogical + 7) >> 3;
    const int logical = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (logical >= a.nlogical) return;
    strip = logical % a.nstrips;
    seg = logical / a.nstrips;
  } else {
    const int x = blockIdx.x & 7;
    const int v = blockIdx.x >> 3;
    const int row = v / a.nstrips;
    strip = v - row * a.nstrips;
    const int i = row / a.ileave, c = row - i * a.ileave;
    const int s0 = x * a.nsegs / 8, s1 = (x + 1) * a.nsegs / 8;
    const int rel = c * a.clen + i;
    if (rel >= s1 - s0) return;
    seg = s0 + rel;
  }

  // the LDS pads are never read into owned results; keep them finite
  for (int j = threadIdx.x; j < RB * 9 * LR; j += LANES) (&s_bfp[0][0][0])[j] = T(0);
  __syncthreads();
  const double pend = MFIX ? hdr->pending : 0.0;
  const double fitmax = MFIX ? hdr->fit_max : 0.0;
  march_tile<T, R, MFIX, STAGE, VARR>(a, n, src, dst, dst2, aux, cf, tabx, taby, uv, part,
                                      pend, fitmax, strip, seg, s_bfp);
}

// Neumaier pair (sum, compensation)
__device__ __forceinline__ void neu_add(double& s, double& c, double v) {
  double t = s + v;
  if (fabs(s) >= fabs(v))
    c += (s - t) + v;
  else
    c += (v - t) + s;
  s = t;
}

// After a step with the fused correction.  The partials hold, per row group,
// the new total M^{n+1} and the number of new cells with f~_0 below
// MASS_FIT_MAX.  A correction below half an ulp of f~_i is lost when it is
// rounded into f~_i, so it goes where it is kept: to those cells (the phase
// with phi near 0), delta = (M0 - M^{n+1}) / count; where fewer than 1 % of
// the cells qualify, to every cell, delta = (M0 - M^{n+1}) / N.  What rounding
// still loses is in the next step's total and corrected then.
// A non-finite total marks the state as blown up (sticky status ENUMERIC) and
// sets no correction.
__device__ __forceinline__ void mass_fix_set(StateHeader* __restrict__ hdr, double m_new,
                                             double nfit, double ncells) {
  const bool to_fit = nfit >= 0.01 * ncells && nfit >= 1.0;
  hdr->fit_max = to_fit ? MASS_FIT_MAX : INFINITY;
  hdr->mass_now = m_new;
  if (isfinite(m_new)) {
    hdr->pending = (hdr->mass0 - m_new) / (to_fit ? nfit : ncells);
  } else {
    hdr->pending = 0.0;
    hdr->status = DUGKS_ENUMERIC;
  }
}

// Fixed-order (Neumaier) sum of n pairs (v[2j], v[2j+1]) by one wavefront:
// lane l takes the pairs l, l + 64, ... (U loads in flight), then the lanes
// are folded in halves.  Lane 0 receives the two totals.  The order depends
// on n only, so any wavefront of any kernel computes the same bits.
__device__ __forceinline__ void wave_pair_sum(const double* __restrict__ v, int n, double& t0,
                                              double& t1) {
  constexpr int U = 8;
  const int lane = threadIdx.x & (LANES - 1);
  double s0 = 0.0, c0 = 0.0, s1 = 0.0, c1 = 0.0;
  for (int j0 = lane; j0 < n; j0 += U * LANES) {
    double w[U][2];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int j = j0 + u * LANES;
      w[u][0] = j < n ? v[2 * j] : 0.0;
      w[u][1] = j < n ? v[2 * j + 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      neu_add(s0, c0, w[u][0]);
      neu_add(s1, c1, w[u][1]);
    }
  }
#pragma unroll
  for (int off = LANES / 2; off > 0; off >>= 1) {
    const double os0 = __shfl_down(s0, off), oc0 = __shfl_down(c0, off);
    const double os1 = __shfl_down(s1, off), oc1 = __shfl_down(c1, off);
    if (lane < off) {
      c0 += oc0;
      neu_add(s0, c0, os0);
      c1 += oc1;
      neu_add(s1, c1, os1);
    }
  }
  t0 = s0 + c0;
  t1 = s1 + c1;
}

// One-grid reduction in one launch: wavefront b sums the groups of strip b
// into strip_part[b]; the last one to finish (counted in the header, with
// device-scope release / acquire around the count) sums the strips in order
// and sets the correction.
static __global__ __launch_bounds__(LANES) void mass_fix_strips_kernel(
    const double* __restrict__ part, int groups_per_strip, int nstrips,
    double* __restrict__ strip_part, StateHeader* __restrict__ hdr, double ncells) {
  double a, b;
  wave_pair_sum(part + 2 * (int64_t)blockIdx.x * groups_per_strip, groups_per_strip, a, b);
  int last = 0;
  if (threadIdx.x == 0) {
    strip_part[2 * blockIdx.x] = a;
    strip_part[2 * blockIdx.x + 1] = b;
    __threadfence();
    last = atomicAdd(&hdr->fix_count, 1) == nstrips - 1;
  }
  last = __shfl(last, 0);
  if (!last) return;
  __threadfence();
  wave_pair_sum(strip_part, nstrips, a, b);
  if (threadIdx.x == 0) {
    mass_fix_set(hdr, a, b, ncells);
    hdr->fix_count = 0;
  }
}

// The same sums by one block for one grid of a batch: its wavefronts take
// the strips in turn, wavefront 0 then sums the strips.
__device__ __forceinline__ void mass_fix_block(const double* __restrict__ part,
                                               int groups_per_strip, int nstrips,
                                               double* __restrict__ strip_part,
                                               StateHeader* __restrict__ hdr, double ncells) {
  const int wave = threadIdx.x / LANES, nwaves = blockDim.x / LANES;
  for (int st = wave; st < nstrips; st += nwaves) {
    double a, b;
    wave_pair_sum(part + 2 * (int64_t)st * groups_per_strip, groups_per_strip, a, b);
    if ((threadIdx.x & (LANES - 1)) == 0) {
      strip_part[2 * st] = a;
      strip_part[2 * st + 1] = b;
    }
  }
  __syncthreads();
  if (wave == 0) {
    double a, b;
    wave_pair_sum(strip_part, nstrips, a, b);
    if (threadIdx.x == 0) mass_fix_set(hdr, a, b, ncells);
  }
}

// ------------------------------------------------------------------ batch
// Many independent grids (slots) advanced together by one persistent kernel.
// Each slot has a descriptor (its scalars and buffers, written by the host when
// the slot is attached) and a step counter pair (n, target) that the finish
// kernel advances; a grid with n >= target is idle.  The work list holds one
// item per (slot, tile) -- tile = seg * nstrips + strip, with the slot's own
// segment height -- and wavefronts take items from queue heads in device
// memory (one queue per XCD, see NQUEUE) until the list is exhausted.
template <typename T>
struct GridDesc {
  StepArgs<T> a;      // T2, or T3S3 stage A
  StepArgs<T> b;      // T3S3 stage B
  T* buf[2];
  T* mid;             // T3S3: f~ at t + dt/3 (stage A -> B)
  T* q;               // T3S3: Q (stage A -> B)
  const T* cf2;       // T3S3: stage B's stencil table
  const T* cf;
  const T* tabx;
  const T* taby;
  StateHeader* hdr;
  double* part;       // row-group partials of the fused mass correction
  double* strip_part; // their per-strip totals
  double ncells;
  int groups_per_strip;
  int nstrips;
};

struct SlotStep {
  int64_t n;          // the step the slot's state is at
  int64_t target;     // the slot stops once n reaches it
};

struct BatchItem {
  int32_t slot, tile;
};

// The work list is cut into up to NQUEUE queues, one per XCD: consecutive
// blocks of a launch go round-robin to the 8 XCDs, so block b drains queue
// b % nq first, and the tiles that share halo rows and columns (one grid's
// neighbouring strips and segments, kept together in one queue) meet in one
// L2.  A block whose own queue is drained takes items from the others.
constexpr int NQUEUE = 8;
// Queue q keeps its heads (stage A or T2, then stage B) in a 128-byte line of
// its own: atomics from different XCDs on one line run several times slower.
constexpr int HEAD_STRIDE = 32;
constexpr size_t HEAD_BYTES = NQUEUE * HEAD_STRIDE * sizeof(unsigned);

struct BatchCtl {
  const BatchItem* items;
  int32_t nitems;
  int32_t nq;                    // queues in use, 1..NQUEUE
  int32_t qstart[NQUEUE + 1];    // queue q holds items [qstart[q], qstart[q + 1])
};

// One batch step (STAGE_T2), or one stage of a T3S3 batch step, over the work
// list; the two T3S3 stages take their items from separate queue heads.
template <typename T, int R, bool MFIX, int STAGE = STAGE_T2>
__global__ __launch_bounds__(LANES, step_waves(sizeof(T), R, MFIX)) void batch_step_kernel(
    const GridDesc<T>* __restrict__ desc, const SlotStep* __restrict__ steps,
    const BatchCtl* __restrict__ ctl, unsigned* __restrict__ head) {
  constexpr int RB = Marcher<T, R, MFIX, STAGE>::RB;
  constexpr int LR = lrow(R);
  __shared__ T s_bfp[RB][9][LR];
  for (int j = threadIdx.x; j < RB * 9 * LR; j += LANES) (&s_bfp[0][0][0])[j] = T(0);
  __syncthreads();
  // descriptors, counters and the work list are not written while the kernel
  // runs: uniform reads through the scalar cache
  const cptr<BatchCtl> c = as_const(ctl);
  const cptr<BatchItem> items = as_const(c->items);
  const cptr<SlotStep> st = as_const(steps);
  const int nq = c->nq;
  const int home = nq > 0 ? (int)(blockIdx.x % (unsigned)nq) : 0;
  unsigned* heads = head + (STAGE == STAGE_B ? 1 : 0);
  for (int qi = 0; qi < nq; qi++) {
    const int q = home + qi < nq ? home + qi : home + qi - nq;
    const unsigned lo = (unsigned)c->qstart[q];
    const unsigned cnt = (unsigned)c->qstart[q + 1] - lo;
    unsigned* qh = heads + q * HEAD_STRIDE;
    for (;;) {
      unsigned it = 0;
      if (threadIdx.x == 0) it = atomicAdd(qh, 1u);
      it = __builtin_amdgcn_readfirstlane(it);
      if (it >= cnt) break;
      const BatchItem w = load_const(items + lo + it);
      const int64_t n = st[w.slot].n;
      if (n >= st[w.slot].target) continue;
      const cptr<GridDesc<T>> d = as_const(desc) + w.slot;
      const StepArgs<T> a = load_const(as_const(STAGE == STAGE_B ? &d->b : &d->a));
      const int strip = w.tile % a.nstrips;
      const int seg = w.tile / a.nstrips;
      const int b = (int)(n & 1);
      const double pend = MFIX ? d->hdr->pending : 0.0;
      const double fitmax = MFIX ? d->hdr->fit_max : 0.0;
      if (STAGE == STAGE_T2)
        march_tile<T, R, MFIX, STAGE>(a, n, d->buf[b], d->buf[b ^ 1], nullptr, nullptr, d->cf,
                                      d->tabx, d->taby, nullptr, d->part, pend, fitmax, strip, seg,
                                      s_bfp);
      else if (STAGE == STAGE_A)   // f^^n -> f~(t'), Q
        march_tile<T, R, MFIX, STAGE>(a, n, d->buf[b], d->mid, d->q, nullptr, d->cf, d->tabx,
                                      d->taby, nullptr, d->part, pend, fitmax, strip, seg, s_bfp);
      else                         // f~(t'), Q -> f^^{n+1}
        march_tile<T, R, MFIX, STAGE>(a, n, d->mid, d->buf[b ^ 1], nullptr, d->q, d->cf2,
                                      d->tabx, d->taby, nullptr, d->part, pend, fitmax, strip, seg,
                                      s_bfp);
      // the next item's ring starts from its own rows; order this tile's LDS
      // reads before them
      wave_sync();
    }
  }
}

// After each batch step: per active slot, the fused mass correction (MFIX)
// and n += 1; block 0 rewinds the work queues for the next step.
// A slot whose state reports a non-finite total (status ENUMERIC: from its
// first state, or from this step's fused correction) stops here: its target
// becomes the step it has reached, and the status is kept for the caller.
template <typename T, bool MFIX>
__global__ __launch_bounds__(FIX_THREADS) void batch_finish_kernel(
    const GridDesc<T>* __restrict__ desc, SlotStep* __restrict__ steps,
    unsigned* __restrict__ head, int32_t* __restrict__ status) {
  const int slot = blockIdx.x;
  if (slot == 0 && threadIdx.x < 2 * NQUEUE)   // every queue head, both stages
    head[(threadIdx.x >> 1) * HEAD_STRIDE + (threadIdx.x & 1)] = 0u;
  const int64_t n = steps[slot].n;
  if (n >= steps[slot].target) return;
  const GridDesc<T>& d = desc[slot];
  if (MFIX) {
    mass_fix_block(d.part, d.groups_per_strip, d.nstrips, d.strip_part, d.hdr, d.ncells);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int32_t st = d.hdr->status;
    status[slot] = st;
    steps[slot].n = n + 1;
    if (st != DUGKS_OK) steps[slot].target = n + 1;
  }
}

// ------------------------------------------------------------------ init
template <typename T>
struct InitArgs {
  const double* __restrict__ phi0;  // [ny][nx] dense
  T* __restrict__ buf;              // strip chunks: f~^0 and phi history
  const T* __restrict__ tabx;
  const T* __restrict__ taby;
  const T* __restrict__ uv;         // caller-supplied cell velocities, or nullptr
  Tiling tl;
  double shift, kth;   // stored = feq - shift S (dt/2: f~ of T2, dt/4: f^ of T3S3)
};

// caller-supplied cell velocities (FP64, u plane then v plane) into the state
// in its precision
template <typename T>
__global__ __launch_bounds__(256) void velocity_store_kernel(const double* __restrict__ in,
                                                             T* __restrict__ out, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = T(in[j]);
}

// f~^0 = feq(phi0, u(x,0)) - (dt/2) S^0 with d(phi u)/dt = 0
template <typename T>
__global__ __launch_bounds__(256) void init_kernel(InitArgs<T> a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  const int nx = a.tl.nx, ny = a.tl.ny;
  if (x >= nx || y >= ny) return;
  auto P = [&](int dx, int dy) {
    return a.phi0[(int64_t)wrapi(y + dy, ny) * nx + wrapi(x + dx, nx)];
  };
  const double pC = P(0, 0);
  const double gx = (P(1, 0) - P(-1, 0)) / 3.0 +
                    ((P(1, 1) - P(-1, 1)) + (P(1, -1) - P(-1, -1))) / 12.0;
  const double gy = (P(0, 1) - P(0, -1)) / 3.0 +
                    ((P(1, 1) - P(1, -1)) + (P(-1, 1) - P(-1, -1))) / 12.0;
  const double gm = sqrt(gx * gx + gy * gy);
  const double den = gm > NORMAL_EPS ? gm : NORMAL_EPS;
  const double th = a.kth * pC * (1.0 - pC);
  const double nvx = gx / den, nvy = gy / den;
  double u, v;
  if (a.uv) {
    const int64_t o = (int64_t)y * nx + x;
    u = (double)a.uv[o];
    v = (double)a.uv[(int64_t)nx * ny + o];
  } else {
    u = (double)a.tabx[2 * x + 1] * (double)a.taby[2 * y + 1];
    v = (double)a.tabx[(2 * nx + 2) + 2 * x + 1] * (double)a.taby[(2 * ny + 2) + 2 * y + 1];
  }
#pragma unroll
  for (int i = 0; i < 9; i++) {
    const double eu = ex(i) * u + ey(i) * v;
    const double en = ex(i) * nvx + ey(i) * nvy;
    const double feq = wq(i) * pC * (1.0 + 3.0 * eu);
    const double src = wq(i) * th * en;
    a.buf[a.tl.idx(i, y, x)] = T(feq - a.shift * src);
  }
  a.buf[a.tl.idx(9, y, x)] = T(pC);
}

// ------------------------------------------------------------------ phi
// f~_i of the state: the stored value, plus the pending correction w_i delta
// if the cell's stored f~_0 is below the header's fit_max, rounded as the step
// kernel rounds it when it loads the value
template <typename T>
__device__ __forceinline__ T stored_f(T v, int i, T f0, const StateHeader* hdr) {
  const double pend = hdr->pending;
  return (pend != 0.0 && f0 < T(hdr->fit_max)) ? v + T(wq(i) * pend) : v;
}

template <typename T>
__global__ __launch_bounds__(256) void phi_kernel(const T* __restrict__ buf, Tiling tl,
                                                  const StateHeader* __restrict__ hdr,
                                                  T* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= tl.nx || y >= tl.ny) return;
  const int64_t o = tl.idx(0, y, x);
  const T f0 = buf[o];
  T s = stored_f(f0, 0, f0, hdr);
#pragma unroll
  for (int i = 1; i < 9; i++) s += stored_f(buf[o + i * OWN], i, f0, hdr);
  out[(int64_t)y * tl.nx + x] = s;
}

// the phi history plane (phi^{n-1} of a state at step n), as stored
template <typename T>
__global__ __launch_bounds__(256) void history_kernel(const T* __restrict__ buf, Tiling tl,
                                                      T* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= tl.nx || y >= tl.ny) return;
  out[(int64_t)y * tl.nx + x] = buf[tl.idx(9, y, x)];
}

template <typename T>
__global__ __launch_bounds__(256) void export_kernel(const T* __restrict__ buf, Tiling tl,
                                                     const StateHeader* __restrict__ hdr,
                                                     T* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  const int i = blockIdx.z;
  if (x >= tl.nx || y >= tl.ny) return;
  out[((int64_t)i * tl.ny + y) * tl.nx + x] =
      stored_f(buf[tl.idx(i, y, x)], i, buf[tl.idx(0, y, x)], hdr);
}

// ------------------------------------------------------------------ mass

// block partials of sum(phi) over a fixed cell partition: partial b covers the
// cells b, b + MASS_BLOCKS*MASS_THREADS, ... of thread order; every reduction
// order is fixed, so the result is bitwise reproducible.  STATE: phi = sum of
// the 9 distributions in strip chunks; otherwise a dense [ny][nx] FP64 field.
template <typename T, bool STATE>
__global__ __launch_bounds__(MASS_THREADS) void mass_partial_kernel(
    const T* __restrict__ f, Tiling tl, const StateHeader* __restrict__ hdr,
    double* __restrict__ part) {
  __shared__ double ss[MASS_THREADS], sc[MASS_THREADS];
  const int nx = tl.nx;
  const int64_t N = (int64_t)nx * tl.ny;
  double s = 0.0, c = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * MASS_THREADS + threadIdx.x; j < N;
       j += (int64_t)MASS_BLOCKS * MASS_THREADS) {
    const int y = (int)(j / nx), x = (int)(j % nx);
    double v;
    if (STATE) {
      const int64_t o = tl.idx(0, y, x);
      const T f0 = f[o];
      v = (double)stored_f(f0, 0, f0, hdr);
#pragma unroll
      for (int i = 1; i < 9; i++) v += (double)stored_f(f[o + i * OWN], i, f0, hdr);
    } else {
      v = (double)f[j];
    }
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

// the total, to out (and out2); a non-finite total sets the state's sticky
// status ENUMERIC
static __global__ __launch_bounds__(64) void mass_final_kernel(const double* __restrict__ part,
                                                        double* __restrict__ out,
                                                        double* __restrict__ out2,
                                                        StateHeader* __restrict__ hdr) {
  if (threadIdx.x != 0) return;
  double s = 0.0, c = 0.0;
  for (int b = 0; b < MASS_BLOCKS; b++) {
    c += part[2 * b + 1];
    neu_add(s, c, part[2 * b]);
  }
  const double m = s + c;
  *out = m;
  if (out2) *out2 = m;
  if (!isfinite(m)) hdr->status = DUGKS_ENUMERIC;
}

// f~_i += w_i (M0 - M) / (nx ny)
template <typename T>
__global__ __launch_bounds__(256) void mass_correct_kernel(
    T* __restrict__ buf, Tiling tl, const StateHeader* __restrict__ hdr) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= tl.nx || y >= tl.ny) return;
  const double delta = (hdr->mass0 - hdr->mass_now) / ((double)tl.nx * (double)tl.ny);
  const int64_t o = tl.idx(0, y, x);
#pragma unroll
  for (int i = 0; i < 9; i++) {
    T& f = buf[o + i * OWN];
    f = T((double)f + wq(i) * delta);
  }
}

}  // namespace dugks
