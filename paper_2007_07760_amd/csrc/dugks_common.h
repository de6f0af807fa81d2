// dugks_common.h -- constants, stencil geometry and state layout shared by
// the host and device code of the library (not by the oracle).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "dugks.h"

namespace dugks {

// ------------------------------------------------------------- D2Q9 lattice
// Paper order (Sec. II.B.2): rest, E, NE, N, NW, W, SW, S, SE; xi_i = e_i
// because sqrt(3RT) = 1 with RT = 1/3.
__host__ __device__ constexpr int ex(int i) {
  return (i == 1 || i == 2 || i == 8) ? 1 : ((i == 4 || i == 5 || i == 6) ? -1 : 0);
}
__host__ __device__ constexpr int ey(int i) {
  return (i == 2 || i == 3 || i == 4) ? 1 : ((i == 6 || i == 7 || i == 8) ? -1 : 0);
}
__host__ __device__ constexpr double wq(int i) {
  return i == 0 ? 4.0 / 9.0 : ((i & 1) ? 1.0 / 9.0 : 1.0 / 36.0);
}

// ------------------------------------------------------ stencil geometry
// Face reconstruction bf_i = sum_t c[o][i][t] * fbar+_i(L + (dx_t, dy_t)),
// with L the cell on the low side of the face.  o = 0: east face of L (normal
// +x); o = 1: north face of L (normal +y).  s = offset along the face normal,
// q = offset along the tangent, both from L.  Patch of offsets:
//   central-2, upwind-3, central-4 (narrow): s in [-1, 2], q in [-2, 2]
//     o = 0: dx in [-1, 2], dy in [-2, 2]    o = 1: dx in [-2, 2], dy in [-1, 2]
//   upwind-5 (wide):                         s in [-2, 3], q in [-2, 2]
//     o = 0: dx in [-2, 3], dy in [-2, 2]    o = 1: dx in [-2, 2], dy in [-2, 3]
constexpr int NTAP = 30;   // the most taps of any patch (arrays are sized for it)
__host__ __device__ constexpr bool wide(int recon) { return recon == DUGKS_UPWIND5; }
__host__ __device__ constexpr int ntap(int recon) { return wide(recon) ? 30 : 20; }
__host__ __device__ constexpr int tap_dx(int recon, int o, int t) {
  return wide(recon) ? (o == 0 ? (t % 6) - 2 : (t % 5) - 2)
                     : (o == 0 ? (t % 4) - 1 : (t % 5) - 2);
}
__host__ __device__ constexpr int tap_dy(int recon, int o, int t) {
  return wide(recon) ? (o == 0 ? (t / 6) - 2 : (t / 5) - 2)
                     : (o == 0 ? (t / 4) - 2 : (t / 5) - 1);
}
__host__ __device__ constexpr int tap_index(int recon, int o, int dx, int dy) {
  return wide(recon) ? (o == 0 ? (dy + 2) * 6 + (dx + 2) : (dy + 2) * 5 + (dx + 2))
                     : (o == 0 ? (dy + 2) * 4 + (dx + 1) : (dy + 1) * 5 + (dx + 2));
}

// Which taps a reconstruction uses (compile-time in the kernels).
__host__ __device__ constexpr bool tap_used(int recon, int o, int i, int t) {
  int dx = tap_dx(recon, o, t), dy = tap_dy(recon, o, t);
  int s = o == 0 ? dx : dy;
  int q = o == 0 ? dy : dx;
  int en = o == 0 ? ex(i) : ey(i);
  int et = o == 0 ? ey(i) : ex(i);
  if (recon == DUGKS_UPWIND5) {
    // five cells centred on the upstream cell along the normal (six centred on
    // the face when en = 0), five along the tangent (one when et = 0)
    int lo = en < 0 ? -1 : -2;
    int hi = en > 0 ? 2 : 3;
    return s >= lo && s <= hi && (et != 0 || q == 0);
  }
  if (recon == DUGKS_UPWIND3) {
    int lo = en < 0 ? 0 : -1;   // upstream cell L (s=0) or R (s=1), 3x3 about it
    int hi = en > 0 ? 1 : 2;
    return s >= lo && s <= hi && q >= -1 && q <= 1;
  }
  if (recon == DUGKS_CENTRAL2)
    return (s == 0 || s == 1) && (q == 0 || (et != 0 && (q == 1 || q == -1)));
  // CENTRAL4
  return s >= -1 && s <= 2 && (q == 0 || et != 0);
}

// ------------------------------------------------ compact coefficient table
// The stencil of (orientation o, velocity i) depends only on the velocity's
// components along the face normal and tangent, en = e_i.n and et = e_i.t, and
// the lattice's mirror symmetries relate the signs: mirroring across the face
// (s -> 1 - s) maps en -> -en, mirroring across the normal (q -> -q) maps
// et -> -et.  So four classes (|en|, |et|) hold every coefficient, in canonical
// tap coordinates s' = (en < 0 ? 1 - s : s), q' = (et < 0 ? -q : q), further
// folded where a class is symmetric: q' -> |q'| when et = 0 (even in q) and
// s' -> min(s', 1 - s') when en = 0 (even about the face).  The mirrors are
// exact symmetries of every scheme here, so no entry changes sign.
//
// Compact layout: class c = 2|en| + |et|, entry (s', q') at
//   c * cclass + (s' - smin) * 5 + (q' + 2),   q' in [-2, 2],
// s' in [-1, 2] (narrow patch, smin = -1, cclass = 20) or [-2, 3] (wide,
// smin = -2, cclass = 30).
constexpr int NCOMPACT = 4 * 30;  // slots for the widest patch
__host__ __device__ constexpr int cclass(int recon) { return wide(recon) ? 30 : 20; }
__host__ __device__ constexpr int cls_of(int en, int et) {
  return 2 * (en < 0 ? -en : en) + (et < 0 ? -et : et);
}
__host__ __device__ constexpr int canon_s(int en, int s) {
  return en < 0 ? 1 - s : (en == 0 ? (s < 1 - s ? s : 1 - s) : s);
}
__host__ __device__ constexpr int canon_q(int et, int q) {
  return et < 0 ? -q : (et == 0 ? (q < 0 ? -q : q) : q);
}
// compact index of tap t of (o, i)
__host__ __device__ constexpr int compact_index(int recon, int o, int i, int t) {
  int dx = tap_dx(recon, o, t), dy = tap_dy(recon, o, t);
  int s = o == 0 ? dx : dy;
  int q = o == 0 ? dy : dx;
  int en = o == 0 ? ex(i) : ey(i);
  int et = o == 0 ? ey(i) : ex(i);
  return cls_of(en, et) * cclass(recon) + (canon_s(en, s) + (wide(recon) ? 2 : 1)) * 5 +
         (canon_q(et, q) + 2);
}

// ------------------------------------------------------------- march tiles
// One wavefront owns a strip of OWN columns and marches up a segment of rows.
// Its 64 lanes hold columns x0-3 .. x0+60: 3 halo columns each side.
constexpr int LANES = 64;
constexpr int HALO = 3;
constexpr int OWN = LANES - 2 * HALO;
// LDS row padding each side (the taps reach 2 columns past a lane, 3 for the
// wide patch) and LDS row length, in elements
__host__ __device__ constexpr int lpad(int recon) { return wide(recon) ? 3 : 2; }
__host__ __device__ constexpr int lrow(int recon) { return LANES + 2 * lpad(recon); }


// Wavefronts per SIMD the step kernels are built for (the register budget of
// each variant: 512 / waves VGPRs), and so resident per CU (x 4 SIMDs).  The
// FP32 variants with the fused mass correction or the 5-row ring of central-4
// need more than 128 registers: 3.
// Upwind-5 (wide patch, 6-row ring, the edge lanes' extra column): 1 (FP64,
// whose ring lets at most 5 wavefronts share a CU's LDS anyway) and 2 (FP32).
__host__ __device__ constexpr int step_waves(int esize, int recon, bool mfix) {
  return wide(recon) ? (esize == 8 ? 1 : 2)
                     : (esize == 8 ? 2 : ((recon == DUGKS_CENTRAL4 || mfix) ? 3 : 4));
}

// ------------------------------------------------------------- state layout
// The distributions live in strip chunks: the grid is cut into strips of OWN
// columns (the columns one wavefront owns), and row y of strip s holds the 9
// planes of f~ and the phi history plane (plane 9) of its OWN columns in one
// contiguous chunk, padded to whole 128-byte lines:
//     element (i, y, x) at ((x / OWN) * ny + y) * CH + i * OWN + x % OWN.
// A wavefront's row then reads one contiguous chunk (plus 3-column halo
// slivers of the neighbour strips) and writes whole cache lines.
constexpr int NPLANE = 10;          // 9 distributions + phi history
struct Tiling {
  int nx, ny, nstrips;
  int64_t CH;                       // chunk length (elements)
  __host__ __device__ int64_t idx(int i, int y, int x) const {
    const int s = x / OWN;
    return ((int64_t)s * ny + y) * CH + (int64_t)i * OWN + (x - s * OWN);
  }
};

// [header 256 B][coef table][coef table 2][x tables][y tables][buffer A][buffer B]
// [T3S3: mid buffer, Q buffer][mass scratch][row-group and strip mass partials]
struct StateHeader {
  uint64_t magic;
  double mass0;        // FP64 total of phi0
  double mass_now;     // last measured total
  double pending;      // fused correction: f~_i = stored f~_i + w_i pending
  int32_t nx, ny, precision, recon;
  double fit_max;      // fused correction: cells with stored f~_0 below it take it
  int32_t fix_count;   // fused correction: strips reduced so far in this step
  int32_t status;      // DUGKS_OK, or DUGKS_ENUMERIC once a non-finite total was seen
  int64_t pad[24];
};
static_assert(sizeof(StateHeader) == 256, "header size");
constexpr uint64_t STATE_MAGIC = 0x53474B5547554431ull;  // "1DUGUKGS"

constexpr int MASS_BLOCKS = 256;   // fixed partial count: deterministic order
constexpr int MASS_THREADS = 256;
// The fused mass correction sums phi^{n+1} in groups of MASS_GROUP rows of one
// strip; segments of such plans are whole groups.
constexpr int MASS_GROUP = 8;
// the fused correction goes to the cells with f~_0 below this (phi below
// ~2e-3), where it is far above half an ulp of every f~_i
constexpr double MASS_FIT_MAX = 1e-3;
constexpr int FIX_THREADS = 1024;   // threads of the block that reduces the groups

// The unit normal of Eq. (2): n = g / max(|g|, NORMAL_EPS), g the isotropic
// gradient of phi (n = 0 where phi is exactly flat).
constexpr double NORMAL_EPS = 1e-12;

struct Layout {
  size_t esize;        // bytes per element (8 or 4)
  Tiling tl;
  size_t off_coef, off_coef2, off_tabx, off_taby, off_vel, off_buf[2], off_mid, off_q;
  size_t off_scratch, off_groups, off_strips, total;
  int ngroups;         // row groups per strip
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline Layout make_layout(int nx, int ny, int precision, int scheme, int vel_kind) {
  Layout L;
  L.esize = precision == DUGKS_F64 ? 8 : 4;
  const int64_t line = 128 / (int64_t)L.esize;
  L.tl.nx = nx;
  L.tl.ny = ny;
  L.tl.nstrips = (nx + OWN - 1) / OWN;
  L.tl.CH = (NPLANE * OWN + line - 1) / line * line;
  const size_t buf_elems = (size_t)L.tl.nstrips * ny * L.tl.CH;
  size_t off = sizeof(StateHeader);
  L.off_coef = off;
  off = align_up(off + NCOMPACT * L.esize, 256);
  L.off_coef2 = off;
  off = align_up(off + NCOMPACT * L.esize, 256);
  L.off_tabx = off;
  off = align_up(off + 2 * (2 * (size_t)nx + 2) * L.esize, 256);
  L.off_taby = off;
  off = align_up(off + 2 * (2 * (size_t)ny + 2) * L.esize, 256);
  // caller-supplied cell velocities (DUGKS_VEL_ARRAYS): u plane, v plane,
  // [ny][nx] dense in the plan's precision
  L.off_vel = 0;
  if (vel_kind == DUGKS_VEL_ARRAYS) {
    L.off_vel = off;
    off = align_up(off + 2 * (size_t)nx * ny * L.esize, 256);
  }
  for (int b = 0; b < 2; b++) {
    L.off_buf[b] = off;
    off = align_up(off + buf_elems * L.esize, 256);
  }
  L.off_mid = L.off_q = 0;
  if (scheme == DUGKS_T3S3) {
    L.off_mid = off;
    off = align_up(off + buf_elems * L.esize, 256);
    L.off_q = off;
    off = align_up(off + buf_elems * L.esize, 256);
  }
  L.off_scratch = off;
  off = align_up(off + 2 * MASS_BLOCKS * sizeof(double) + 64, 256);
  L.ngroups = (ny + MASS_GROUP - 1) / MASS_GROUP;
  L.off_groups = off;
  off = align_up(off + 2 * (size_t)L.tl.nstrips * L.ngroups * sizeof(double), 256);
  L.off_strips = off;
  off = align_up(off + 2 * (size_t)L.tl.nstrips * sizeof(double), 256);
  L.total = off;
  return L;
}

}  // namespace dugks
