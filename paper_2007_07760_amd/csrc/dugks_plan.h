// dugks_plan.h -- the plan object and the launch helpers shared by the
// single-grid and batch entry points (private to the library).
#pragma once

#include <math.h>

#include <mutex>
#include <vector>

#include "dugks_common.h"
#include "dugks_kernels.h"

struct dugks_plan {
  dugks_params p;
  dugks::Layout L;
  double coef[2][9][dugks::NTAP];   // face stencils (Eqs. 25-26)
  double compact[dugks::NCOMPACT];  // the same, folded by the lattice symmetries
  double dt, h, tau;
  double cA, cB, cA2, cB2, alpha, beta, gamma;
  double period;             // cos(pi t / period) modulation; 0 = steady
  // coefficients of each launch kind (dugks::Stage): the face stencil is built
  // with the stage's half step h; fbar+ = g + cbar (X - g) from the stage's
  // input g; the outputs take kap (X - fbar+) and wo1 / wo2 dt L; d(phi u)/dt
  // uses phi at n dt + toff and at n dt + troff
  struct StageCoef {
    double h, cbar, kap, wo1, wo2, alpha, beta, gamma, toff, troff, jdt;
    int jfirst;
  } st[3];
  double compact2[dugks::NCOMPACT];  // T3S3 stage B stencil (compact: stage A)
  int seg_rows, nstrips, nsegs;
  std::vector<double> tabx, taby;
  // the constant head of every state of this plan (header, coefficient and
  // velocity tables in the plan's precision), staged once in pinned host memory
  // so that dugks_init can copy it asynchronously
  mutable std::once_flag staged;
  mutable void* head = nullptr;
  mutable int head_rc = DUGKS_OK;
};

namespace dugks {

inline int hip_status(hipError_t e) { return e == hipSuccess ? DUGKS_OK : DUGKS_EDEVICE; }

template <typename T>
inline T* at(void* state, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(state) + off);
}
template <typename T>
inline const T* at(const void* state, size_t off) {
  return reinterpret_cast<const T*>(static_cast<const char*>(state) + off);
}

inline bool aligned(const void* ptr) { return ((uintptr_t)ptr & 255u) == 0; }


template <typename T>
inline StepBufs<T> step_bufs(const dugks_plan* P, void* state, int64_t n) {
  const Layout& L = P->L;
  const int b = (int)(n & 1);
  StepBufs<T> q;
  q.src = at<T>(state, L.off_buf[b]);
  q.dst = at<T>(state, L.off_buf[b ^ 1]);
  q.cf = at<T>(state, L.off_coef);
  q.tabx = at<T>(state, L.off_tabx);
  q.taby = at<T>(state, L.off_taby);
  return q;
}

template <typename T>
inline StepArgs<T> step_args(const dugks_plan* P, int stage = STAGE_T2) {
  const Layout& L = P->L;
  StepArgs<T> a;
  a.CH = L.tl.CH;
  a.nx = P->p.nx;
  a.ny = P->p.ny;
  a.seg_rows = P->seg_rows;
  a.nstrips = P->nstrips;
  a.nsegs = P->nsegs;
  a.nlogical = P->nstrips * P->nsegs;
  // interleave two chunks of each XCD's band once it holds 4 segments or more
  // (not for the wide patch: one wavefront per SIMD, and it measured slower)
  a.ileave = P->nsegs >= 32 && !wide(P->p.recon) ? 2 : 1;
  a.clen = ((P->nsegs + 7) / 8 + a.ileave - 1) / a.ileave;
  a.ngroups = L.ngroups;
  const dugks_plan::StageCoef& c = P->st[stage];
  a.cB2 = T(c.cbar);
  a.kap = T(c.kap);
  a.wo1 = T(c.wo1);
  a.wo2 = T(c.wo2);
  a.pscale = T(c.beta / c.alpha);
  a.gdt = T(0.5 * P->dt * c.gamma);
  a.dt = T(P->dt);
  a.jinv = T(1) / T(c.jdt);
  a.toff = c.toff;
  a.troff = c.troff;
  a.jfirst = c.jfirst;
  a.tau = T(P->tau);
  a.kth = isfinite(P->p.width) ? T(4.0 / P->p.width) : T(0);
  a.period = P->period;
  a.dtd = P->dt;
  a.hd = c.h;
  a.jzero = (P->p.flags & DUGKS_FLAG_DTPHIU_ZERO) ? 1 : 0;
  return a;
}

}  // namespace dugks
