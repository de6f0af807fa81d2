// dugks_batch_impl.h -- pieces of the batch path shared by the batch entry
// points and the allocation-free multi-grid step (private to the library).
#pragma once

#include <string.h>

#include <algorithm>

#include "dugks_common.h"
#include "dugks_kernels.h"
#include "dugks_plan.h"

namespace dugks {

// Device memory one batch step works on: descriptors, step counters, slot
// status, the work-list control block and the queue heads.
struct BatchDev {
  const void* desc;
  SlotStep* steps;
  int32_t* status;
  BatchCtl* ctl;
  unsigned* head;
  int nslots;        // finish-kernel blocks (one per slot)
  int grid_blocks;   // resident wavefronts of the persistent kernel
};

// One batch step (finish = true) or the step kernels alone, on `s`, for grids
// of one precision / reconstruction / mass-fix flag / time scheme.
int launch_batch(const BatchDev& D, int precision, int recon, bool mfix, int scheme,
                 hipStream_t s, bool finish);

// Resident wavefronts per CU of the batch step kernel of that kind.
int batch_occupancy(int precision, int recon, bool mfix, int scheme, int* per_cu);

// The descriptor of one grid (plan, state), its tiles `rows` high.
template <typename T>
inline GridDesc<T> make_grid_desc(const dugks_plan* P, void* state, int rows) {
  GridDesc<T> d;
  memset(&d, 0, sizeof(d));
  if (!P) return d;
  const Layout& L = P->L;
  const bool t3 = P->p.scheme == DUGKS_T3S3;
  d.a = step_args<T>(P, t3 ? STAGE_A : STAGE_T2);
  d.b = step_args<T>(P, t3 ? STAGE_B : STAGE_T2);
  const int seg = std::min(rows, P->p.ny);
  for (StepArgs<T>* a : {&d.a, &d.b}) {
    a->seg_rows = seg;
    a->nsegs = (P->p.ny + seg - 1) / seg;
    a->nlogical = a->nstrips * a->nsegs;
    a->ileave = 1;   // unused: a batch takes its tiles from its work queues
    a->clen = a->nsegs;
  }
  if (t3) {
    d.mid = at<T>(state, L.off_mid);
    d.q = at<T>(state, L.off_q);
    d.cf2 = at<T>(state, L.off_coef2);
  }
  d.buf[0] = at<T>(state, L.off_buf[0]);
  d.buf[1] = at<T>(state, L.off_buf[1]);
  d.cf = at<T>(state, L.off_coef);
  d.tabx = at<T>(state, L.off_tabx);
  d.taby = at<T>(state, L.off_taby);
  d.hdr = at<StateHeader>(state, 0);
  d.part = at<double>(state, L.off_groups);
  d.ncells = (double)P->p.nx * (double)P->p.ny;
  d.strip_part = at<double>(state, L.off_strips);
  d.groups_per_strip = L.ngroups;
  d.nstrips = L.tl.nstrips;
  return d;
}

}  // namespace dugks
