// dugks_batch.hip -- C ABI of batches (include/dugks.h): many independent
// grids of one precision and reconstruction advanced by one persistent kernel,
// replayed from a captured hipGraph, with a measured choice of tile height.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "dugks_common.h"
#include "dugks_kernels.h"
#include "dugks_plan.h"
#include "dugks_batch_impl.h"

using namespace dugks;

namespace {

constexpr int NSTAGE = 3;   // pinned staging buffers in flight

// Tile heights the autotuner tries (whole mass groups).
constexpr int TUNE_ROWS[] = {16, 24, 32, 48, 64, 96, 128, 192, 256};
constexpr int DEFAULT_ROWS = 64;

struct Slot {
  const dugks_plan* plan = nullptr;
  void* state = nullptr;
  int64_t step = 0, target = 0;
  bool step_dirty = false;
};

}  // namespace

namespace dugks {

template <typename T, int R, bool MFIX>
static int launch_batch_step(const BatchDev& D, int scheme, hipStream_t s, bool finish) {
  const GridDesc<T>* desc = static_cast<const GridDesc<T>*>(D.desc);
  if (scheme == DUGKS_T3S3) {   // the two stages over every tile, in turn
    hipLaunchKernelGGL((batch_step_kernel<T, R, MFIX, STAGE_A>), dim3(D.grid_blocks),
                       dim3(LANES), 0, s, desc, D.steps, D.ctl, D.head);
    hipLaunchKernelGGL((batch_step_kernel<T, R, MFIX, STAGE_B>), dim3(D.grid_blocks),
                       dim3(LANES), 0, s, desc, D.steps, D.ctl, D.head);
  } else {
    hipLaunchKernelGGL((batch_step_kernel<T, R, MFIX>), dim3(D.grid_blocks), dim3(LANES), 0, s,
                       desc, D.steps, D.ctl, D.head);
  }
  if (finish)
    hipLaunchKernelGGL((batch_finish_kernel<T, MFIX>), dim3(D.nslots), dim3(FIX_THREADS), 0, s,
                       desc, D.steps, D.head, D.status);
  return hip_status(hipGetLastError());
}

int launch_batch(const BatchDev& D, int precision, int recon, bool mfix, int scheme,
                 hipStream_t s, bool finish) {
#define DUGKS_BATCH(TT, RR)                                                    \
  return mfix ? launch_batch_step<TT, RR, true>(D, scheme, s, finish)          \
              : launch_batch_step<TT, RR, false>(D, scheme, s, finish)
#define DUGKS_BATCH_R(TT)                                        \
  switch (recon) {                                               \
    case DUGKS_CENTRAL2: DUGKS_BATCH(TT, DUGKS_CENTRAL2);        \
    case DUGKS_UPWIND3: DUGKS_BATCH(TT, DUGKS_UPWIND3);          \
    default: DUGKS_BATCH(TT, DUGKS_CENTRAL4);                    \
  }
  if (precision == DUGKS_F64) {
    DUGKS_BATCH_R(double)
  } else {
    DUGKS_BATCH_R(float)
  }
#undef DUGKS_BATCH_R
#undef DUGKS_BATCH
}

template <typename T, int R, bool MFIX>
static int occupancy(int* per_cu, int scheme) {
  if (scheme == DUGKS_T3S3) {   // the smaller of the two stages' residencies
    int a = 0, b = 0;
    int rc = hip_status(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &a, reinterpret_cast<const void*>(&batch_step_kernel<T, R, MFIX, STAGE_A>), LANES, 0));
    if (!rc)
      rc = hip_status(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &b, reinterpret_cast<const void*>(&batch_step_kernel<T, R, MFIX, STAGE_B>), LANES,
          0));
    *per_cu = std::min(a, b);
    return rc;
  }
  return hip_status(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      per_cu, reinterpret_cast<const void*>(&batch_step_kernel<T, R, MFIX>), LANES, 0));
}

int batch_occupancy(int precision, int recon, bool mfix, int scheme, int* per_cu) {
#define DUGKS_OCC(TT, RR)                                   \
  return mfix ? occupancy<TT, RR, true>(per_cu, scheme)     \
              : occupancy<TT, RR, false>(per_cu, scheme)
#define DUGKS_OCC_R(TT)                                 \
  switch (recon) {                                      \
    case DUGKS_CENTRAL2: DUGKS_OCC(TT, DUGKS_CENTRAL2);  \
    case DUGKS_UPWIND3: DUGKS_OCC(TT, DUGKS_UPWIND3);    \
    default: DUGKS_OCC(TT, DUGKS_CENTRAL4);              \
  }
  if (precision == DUGKS_F64) {
    DUGKS_OCC_R(double)
  } else {
    DUGKS_OCC_R(float)
  }
#undef DUGKS_OCC_R
#undef DUGKS_OCC
}

}  // namespace dugks

struct dugks_batch {
  int cap = 0, precision = 0, recon = 0;
  int scheme = DUGKS_T2;              // every attached plan's time scheme
  bool mfix = false;
  int device = 0;
  size_t desc_bytes = 0;              // sizeof(GridDesc<T>)
  // device memory owned by the batch
  void* d_desc = nullptr;             // GridDesc<T>[cap]
  SlotStep* d_steps = nullptr;        // [cap]
  int32_t* d_status = nullptr;        // [cap] status of each slot's state
  BatchCtl* d_ctl = nullptr;
  unsigned* d_head = nullptr;
  BatchItem* d_items = nullptr;
  size_t items_cap = 0;
  // host side
  std::vector<Slot> slots;
  std::vector<BatchItem> items;
  std::vector<int32_t> qstart;        // queue q: items [qstart[q], qstart[q + 1])
  int nq = 1;
  bool desc_dirty = true;
  int rows = DEFAULT_ROWS;            // tile height (rows per item)
  int grid_blocks = 0;                // resident wavefronts of the persistent kernel
  // pinned staging ring: [ctl][desc table][steps][items]
  void* stage[NSTAGE] = {};
  size_t stage_bytes[NSTAGE] = {};
  hipEvent_t stage_ev[NSTAGE] = {};
  int stage_next = 0;
  // graph of K steps
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_k = 0;
};

namespace {

template <typename T>
GridDesc<T> make_desc(const Slot& s, int rows) {
  return make_grid_desc<T>(s.plan, s.state, rows);
}

// Work list for tile height `rows`, cut into NQUEUE queues of about equal
// work (one per XCD).  The slots' tiles, largest slot first and each slot's
// tiles segment by segment, are laid end to end and cut at equal shares of
// the marched rows, so a queue holds whole small grids or a band of segments
// of a large one: tiles that share halos stay in one XCD's L2.  Within a
// queue the taller tiles come first, so that the short ones fill the tail.
void build_items(dugks_batch* B, int rows) {
  B->items.clear();
  struct Keyed {
    int h;
    BatchItem it;
  };
  std::vector<std::pair<int64_t, int>> order;   // (marched rows, slot)
  for (int k = 0; k < B->cap; k++) {
    const Slot& s = B->slots[k];
    if (!s.plan) continue;
    const int ny = s.plan->p.ny;
    const int seg = std::min(rows, ny);
    const int64_t nsegs = (ny + seg - 1) / seg;
    order.push_back({(int64_t)s.plan->nstrips * (ny + 5 * nsegs), k});
  }
  std::stable_sort(order.begin(), order.end(),
                   [](const std::pair<int64_t, int>& a, const std::pair<int64_t, int>& b) {
                     return a.first > b.first;
                   });
  std::vector<Keyed> v;
  for (const auto& o : order) {
    const int k = o.second;
    const Slot& s = B->slots[k];
    const int ny = s.plan->p.ny, nstrips = s.plan->nstrips;
    const int seg = std::min(rows, ny);
    const int nsegs = (ny + seg - 1) / seg;
    for (int g = 0; g < nsegs; g++) {
      const int h = std::min(seg, ny - g * seg);
      for (int st = 0; st < nstrips; st++) v.push_back({h, {k, g * nstrips + st}});
    }
  }
  int64_t total = 0;
  for (const Keyed& k : v) total += k.h + 5;
  B->nq = v.empty() ? 1 : NQUEUE;
  B->qstart.assign(NQUEUE + 1, (int32_t)v.size());
  B->qstart[0] = 0;
  size_t i = 0;
  int64_t done = 0;
  for (int q = 0; q < B->nq; q++) {
    const size_t first = i;
    // up to the queue's share of the work (the last queue takes the rest)
    const int64_t upto = total * (q + 1) / B->nq;
    while (i < v.size() && (q == B->nq - 1 || done + v[i].h + 5 <= upto)) done += v[i++].h + 5;
    std::stable_sort(v.begin() + first, v.begin() + i,
                     [](const Keyed& a, const Keyed& b) { return a.h > b.h; });
    B->qstart[q + 1] = (int32_t)i;
  }
  B->items.reserve(v.size());
  for (const Keyed& k : v) B->items.push_back(k.it);
}

int ensure_items_cap(dugks_batch* B, size_t n, hipStream_t s) {
  if (n <= B->items_cap) return DUGKS_OK;
  // in-flight steps may still read the old list
  if (hipStreamSynchronize(s) != hipSuccess) return DUGKS_EDEVICE;
  if (B->d_items) (void)hipFree(B->d_items);
  B->d_items = nullptr;
  B->items_cap = 0;
  size_t cap = std::max<size_t>(n, 2 * n);
  if (hipMalloc(&B->d_items, cap * sizeof(BatchItem)) != hipSuccess) return DUGKS_EDEVICE;
  B->items_cap = cap;
  return DUGKS_OK;
}

// Copy the descriptor table, the changed step counters and the work list to
// the device (asynchronous, through the pinned staging ring).
template <typename T>
int upload(dugks_batch* B, hipStream_t s) {
  int rc = ensure_items_cap(B, std::max<size_t>(B->items.size(), 1), s);
  if (rc) return rc;
  const size_t off_desc = 256;
  const size_t off_steps = align_up(off_desc + B->cap * sizeof(GridDesc<T>), 256);
  const size_t off_status = align_up(off_steps + B->cap * sizeof(SlotStep), 256);
  const size_t off_items = align_up(off_status + B->cap * sizeof(int32_t), 256);
  const size_t need = off_items + B->items.size() * sizeof(BatchItem);
  const int j = B->stage_next;
  B->stage_next = (j + 1) % NSTAGE;
  if (hipEventSynchronize(B->stage_ev[j]) != hipSuccess) return DUGKS_EDEVICE;
  if (B->stage_bytes[j] < need) {
    if (B->stage[j]) (void)hipHostFree(B->stage[j]);
    B->stage[j] = nullptr;
    B->stage_bytes[j] = 0;
    if (hipHostMalloc(&B->stage[j], 2 * need, hipHostMallocDefault) != hipSuccess)
      return DUGKS_EDEVICE;
    B->stage_bytes[j] = 2 * need;
  }
  char* h = static_cast<char*>(B->stage[j]);
  BatchCtl* ctl = reinterpret_cast<BatchCtl*>(h);
  ctl->items = B->d_items;
  ctl->nitems = (int32_t)B->items.size();
  ctl->nq = B->nq;
  for (int q = 0; q <= NQUEUE; q++)
    ctl->qstart[q] = q < (int)B->qstart.size() ? B->qstart[q] : ctl->nitems;
  hipError_t e;
  if ((e = hipMemcpyAsync(B->d_ctl, ctl, sizeof(BatchCtl), hipMemcpyHostToDevice, s)))
    return hip_status(e);
  if (B->desc_dirty) {
    GridDesc<T>* dt = reinterpret_cast<GridDesc<T>*>(h + off_desc);
    for (int k = 0; k < B->cap; k++) dt[k] = make_desc<T>(B->slots[k], B->rows);
    if ((e = hipMemcpyAsync(B->d_desc, dt, B->cap * sizeof(GridDesc<T>), hipMemcpyHostToDevice,
                            s)))
      return hip_status(e);
    B->desc_dirty = false;
  }
  SlotStep* st = reinterpret_cast<SlotStep*>(h + off_steps);
  int32_t* ss = reinterpret_cast<int32_t*>(h + off_status);
  for (int k = 0; k < B->cap; k++) {
    Slot& sl = B->slots[k];
    if (!sl.step_dirty) continue;
    st[k].n = sl.step;
    st[k].target = sl.target;
    ss[k] = DUGKS_OK;   // a newly attached (or cleared) slot has no status yet
    if ((e = hipMemcpyAsync(B->d_steps + k, st + k, sizeof(SlotStep), hipMemcpyHostToDevice,
                            s)) ||
        (e = hipMemcpyAsync(B->d_status + k, ss + k, sizeof(int32_t), hipMemcpyHostToDevice, s)))
      return hip_status(e);
    sl.step_dirty = false;
  }
  if (!B->items.empty()) {
    BatchItem* it = reinterpret_cast<BatchItem*>(h + off_items);
    memcpy(it, B->items.data(), B->items.size() * sizeof(BatchItem));
    if ((e = hipMemcpyAsync(B->d_items, it, B->items.size() * sizeof(BatchItem),
                            hipMemcpyHostToDevice, s)))
      return hip_status(e);
  }
  return hip_status(hipEventRecord(B->stage_ev[j], s));
}

// finish = false: the step kernel alone, which writes only the next-step
// buffers and mass partials of each active slot (used to time tilings; the
// state is unchanged, since the finish kernel never runs)
int batch_launch(dugks_batch* B, hipStream_t s, bool finish) {
  const BatchDev D{B->d_desc, B->d_steps, B->d_status, B->d_ctl, B->d_head, B->cap,
                   B->grid_blocks};
  return launch_batch(D, B->precision, B->recon, B->mfix, B->scheme, s, finish);
}

int commit(dugks_batch* B, hipStream_t s) {
  build_items(B, B->rows);
  return B->precision == DUGKS_F64 ? upload<double>(B, s) : upload<float>(B, s);
}

void release(dugks_batch* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
  for (int j = 0; j < NSTAGE; j++) {
    if (B->stage_ev[j]) {
      (void)hipEventSynchronize(B->stage_ev[j]);
      (void)hipEventDestroy(B->stage_ev[j]);
    }
    if (B->stage[j]) (void)hipHostFree(B->stage[j]);
  }
  if (B->d_items) (void)hipFree(B->d_items);
  if (B->d_desc) (void)hipFree(B->d_desc);
  if (B->d_steps) (void)hipFree(B->d_steps);
  if (B->d_status) (void)hipFree(B->d_status);
  if (B->d_ctl) (void)hipFree(B->d_ctl);
  if (B->d_head) (void)hipFree(B->d_head);
}

int capture_graph(dugks_batch* B, int k) {
  if (B->exec && B->graph_k == k) return DUGKS_OK;
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
  if (hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess)
    return DUGKS_EDEVICE;
  int rc = DUGKS_OK;
  for (int j = 0; j < k && rc == DUGKS_OK; j++) rc = batch_launch(B, B->cap_stream, true);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(B->cap_stream, &g);
  if (rc || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return DUGKS_EDEVICE;
  }
  B->graph = g;
  if (hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    B->exec = nullptr;
    return DUGKS_EDEVICE;
  }
  B->graph_k = k;
  return DUGKS_OK;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

int dugks_batch_create(int32_t capacity, int32_t precision, int32_t recon, uint32_t flags,
                       dugks_batch** out) {
  if (!out) return DUGKS_EINVAL;
  *out = nullptr;
  if (capacity < 1 || capacity > 65536 || precision < 0 || precision > 1 || recon < 0 ||
      recon > 3 || (flags & ~(DUGKS_FLAG_MASS_FIX | DUGKS_BATCH_T3S3)))
    return DUGKS_EINVAL;
  if (recon == DUGKS_UPWIND5) return DUGKS_EUNSUPPORTED;   // single grids only
  dugks_batch* B = new (std::nothrow) dugks_batch();
  if (!B) return DUGKS_ENOMEM;
  B->cap = capacity;
  B->precision = precision;
  B->recon = recon;
  B->mfix = (flags & DUGKS_FLAG_MASS_FIX) != 0;
  B->scheme = (flags & DUGKS_BATCH_T3S3) ? DUGKS_T3S3 : DUGKS_T2;
  B->slots.resize(capacity);
  B->desc_bytes = precision == DUGKS_F64 ? sizeof(GridDesc<double>) : sizeof(GridDesc<float>);
  int rc = DUGKS_OK;
  int per_cu = 0, ncu = 0;
  if (hipGetDevice(&B->device) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, B->device) !=
          hipSuccess ||
      (rc = batch_occupancy(B->precision, B->recon, B->mfix, B->scheme, &per_cu)) !=
          DUGKS_OK ||
      per_cu < 1 || ncu < 1 ||
      hipMalloc(&B->d_desc, capacity * B->desc_bytes) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&B->d_steps), capacity * sizeof(SlotStep)) !=
          hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&B->d_status), capacity * sizeof(int32_t)) !=
          hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&B->d_ctl), sizeof(BatchCtl)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&B->d_head), HEAD_BYTES) != hipSuccess ||
      hipMemset(B->d_desc, 0, capacity * B->desc_bytes) != hipSuccess ||
      hipMemset(B->d_steps, 0, capacity * sizeof(SlotStep)) != hipSuccess ||
      hipMemset(B->d_status, 0, capacity * sizeof(int32_t)) != hipSuccess ||
      hipMemset(B->d_ctl, 0, sizeof(BatchCtl)) != hipSuccess ||
      hipMemset(B->d_head, 0, HEAD_BYTES) != hipSuccess ||
      hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    release(B);
    delete B;
    return rc ? rc : DUGKS_EDEVICE;
  }
  for (int j = 0; j < NSTAGE; j++)
    if (hipEventCreateWithFlags(&B->stage_ev[j], hipEventDisableTiming) != hipSuccess) {
      release(B);
      delete B;
      return DUGKS_EDEVICE;
    }
  if (hipDeviceSynchronize() != hipSuccess) {
    release(B);
    delete B;
    return DUGKS_EDEVICE;
  }
  B->grid_blocks = per_cu * ncu;
  *out = B;
  return DUGKS_OK;
}

void dugks_batch_destroy(dugks_batch* batch) {
  if (!batch) return;
  (void)hipDeviceSynchronize();
  release(batch);
  delete batch;
}

int dugks_batch_set(dugks_batch* batch, int32_t slot, const dugks_plan* plan, void* state,
                    int64_t step, int64_t target) {
  if (!batch || slot < 0 || slot >= batch->cap || !plan || !state || !aligned(state) ||
      step < 0 || target < step)
    return DUGKS_EINVAL;
  if (plan->p.precision != batch->precision || plan->p.recon != batch->recon ||
      ((plan->p.flags & DUGKS_FLAG_MASS_FIX) != 0) != batch->mfix ||
      plan->p.scheme != batch->scheme)
    return DUGKS_EINVAL;
  if (plan->p.vel_kind == DUGKS_VEL_ARRAYS) return DUGKS_EUNSUPPORTED;
  Slot& s = batch->slots[slot];
  s.plan = plan;
  s.state = state;
  s.step = step;
  s.target = target;
  s.step_dirty = true;
  batch->desc_dirty = true;
  return DUGKS_OK;
}

int dugks_batch_clear(dugks_batch* batch, int32_t slot) {
  if (!batch || slot < 0 || slot >= batch->cap) return DUGKS_EINVAL;
  Slot& s = batch->slots[slot];
  s = Slot();
  s.step_dirty = true;   // (n, target) = (0, 0): idle
  batch->desc_dirty = true;
  return DUGKS_OK;
}

int dugks_batch_commit(dugks_batch* batch, void* stream) {
  if (!batch) return DUGKS_EINVAL;
  return commit(batch, static_cast<hipStream_t>(stream));
}

int dugks_batch_step(dugks_batch* batch, int64_t nsteps, int32_t graph_steps, void* stream) {
  if (!batch || nsteps < 0 || graph_steps < 0 || graph_steps > 4096) return DUGKS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int64_t left = nsteps;
  if (graph_steps > 1 && nsteps >= graph_steps) {
    int rc = capture_graph(batch, graph_steps);
    if (rc) return rc;
    for (; left >= graph_steps; left -= graph_steps)
      if (hipGraphLaunch(batch->exec, s) != hipSuccess) return DUGKS_EDEVICE;
  }
  for (; left > 0; left--) {
    int rc = batch_launch(batch, s, true);
    if (rc) return rc;
  }
  return DUGKS_OK;
}

int dugks_batch_steps(const dugks_batch* batch, int64_t* out, void* stream) {
  if (!batch || !out) return DUGKS_EINVAL;
  return hip_status(hipMemcpyAsync(out, batch->d_steps, batch->cap * sizeof(SlotStep),
                                   hipMemcpyDefault, static_cast<hipStream_t>(stream)));
}

int dugks_batch_status(const dugks_batch* batch, int32_t* out, void* stream) {
  if (!batch || !out) return DUGKS_EINVAL;
  return hip_status(hipMemcpyAsync(out, batch->d_status, batch->cap * sizeof(int32_t),
                                   hipMemcpyDefault, static_cast<hipStream_t>(stream)));
}

int dugks_batch_tile_rows(const dugks_batch* batch) { return batch ? batch->rows : -1; }

int dugks_batch_set_tile_rows(dugks_batch* batch, int32_t rows) {
  if (!batch || rows < MASS_GROUP || rows > 65536 || rows % MASS_GROUP) return DUGKS_EINVAL;
  batch->rows = rows;
  batch->desc_dirty = true;
  return DUGKS_OK;
}

int dugks_batch_tune(dugks_batch* batch, int32_t reps, int32_t* rows_out, void* stream) {
  if (!batch || reps < 1 || reps > 1000) return DUGKS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return DUGKS_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return DUGKS_EDEVICE;
  }
  int rc = DUGKS_OK;
  float best_ms = -1.0f;
  int best = batch->rows;
  for (int rows : TUNE_ROWS) {
    batch->rows = rows;
    batch->desc_dirty = true;
    if ((rc = commit(batch, s))) break;
    // one untimed pass, then the timed passes
    if ((rc = batch_launch(batch, s, false))) break;
    // the step kernels alone leave the queue heads at their ends: rewind them
    if (hipMemsetAsync(batch->d_head, 0, HEAD_BYTES, s) != hipSuccess) {
      rc = DUGKS_EDEVICE;
      break;
    }
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && rc == DUGKS_OK; r++) {
      rc = batch_launch(batch, s, false);
      if (!rc && hipMemsetAsync(batch->d_head, 0, HEAD_BYTES, s) != hipSuccess)
        rc = DUGKS_EDEVICE;
    }
    (void)hipEventRecord(e1, s);
    if (rc || hipEventSynchronize(e1) != hipSuccess) {
      rc = rc ? rc : DUGKS_EDEVICE;
      break;
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (best_ms < 0.0f || ms < best_ms) {
      best_ms = ms;
      best = rows;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  batch->rows = best;
  batch->desc_dirty = true;
  int rc2 = commit(batch, s);
  if (!rc) rc = rc2;
  if (!rc && rows_out) *rows_out = best;
  return rc;
}

}  // extern "C"
