// dugks_noalloc.hip -- dugks_step_many_noalloc (include/dugks.h): the batch
// step of many grids for callers that cannot allocate device memory.  It runs
// the batch kernels of dugks_batch.hip; what a batch keeps in device memory of
// its own lives here in one fixed file-scope device array per GPU.
#include <string.h>

#include <algorithm>
#include <mutex>

#include "dugks_batch_impl.h"
#include "dugks_common.h"
#include "dugks_kernels.h"
#include "dugks_plan.h"

using namespace dugks;

namespace {

// dugks_step_many_noalloc keeps what a batch keeps in its own device memory --
// descriptors, step counters, slot status, the work list and its control block
// with the queue heads -- in one file-scope device array of NOALLOC_BYTES per
// GPU, filled by small set-up kernels whose inputs travel as kernel arguments
// (no host staging buffer, no allocation).  Layout of the array:
constexpr int NOALLOC_GRIDS = 256;
constexpr size_t NOALLOC_BYTES = size_t(1) << 20;
constexpr size_t NA_CTL = 0, NA_HEAD = 256, NA_STEPS = NA_HEAD + HEAD_BYTES;
constexpr size_t NA_STATUS = NA_STEPS + NOALLOC_GRIDS * sizeof(SlotStep);
constexpr size_t NA_DESC = (NA_STATUS + NOALLOC_GRIDS * sizeof(int32_t) + 255) / 256 * 256;
constexpr size_t NA_ITEMS =
    (NA_DESC + NOALLOC_GRIDS * sizeof(GridDesc<double>) + 255) / 256 * 256;
constexpr int64_t NOALLOC_ITEMS = (int64_t)((NOALLOC_BYTES - NA_ITEMS) / sizeof(BatchItem));
static_assert(sizeof(GridDesc<double>) >= sizeof(GridDesc<float>), "descriptor sizes");
static_assert(sizeof(BatchCtl) <= NA_HEAD - NA_CTL, "control block");
static_assert(NA_STEPS % 256 == 0, "alignment");

// descriptors of up to DESC_CHUNK grids, by value
constexpr int DESC_CHUNK = 8;
template <typename T>
struct DescChunk {
  GridDesc<T> d[DESC_CHUNK];
  SlotStep st[DESC_CHUNK];
  int first, count;
};
static_assert(sizeof(DescChunk<double>) <= 4096, "kernel argument size");

template <typename T>
__global__ __launch_bounds__(64) void noalloc_desc_kernel(DescChunk<T> c, unsigned char* base) {
  const int k = threadIdx.x;
  if (k >= c.count) return;
  GridDesc<T>* desc = reinterpret_cast<GridDesc<T>*>(base + NA_DESC);
  SlotStep* steps = reinterpret_cast<SlotStep*>(base + NA_STEPS);
  int32_t* status = reinterpret_cast<int32_t*>(base + NA_STATUS);
  desc[c.first + k] = c.d[k];
  steps[c.first + k] = c.st[k];
  status[c.first + k] = DUGKS_OK;
}

// the work list: item i belongs to the grid j with start[j] <= i < start[j+1]
// (grids by queue, then in decreasing order of tile height), tile
// i - start[j]; queue q holds items [qstart[q], qstart[q+1]).  One thread
// also writes the control block and rewinds the queue heads
struct ItemStarts {
  int32_t start[NOALLOC_GRIDS + 1];
  int32_t grid[NOALLOC_GRIDS];
  int32_t qstart[NQUEUE + 1];
  int n, nq;
};
static_assert(sizeof(ItemStarts) <= 4096, "kernel argument size");

static __global__ __launch_bounds__(256) void noalloc_items_kernel(ItemStarts a,
                                                                   unsigned char* base) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nitems = a.start[a.n];
  BatchItem* items = reinterpret_cast<BatchItem*>(base + NA_ITEMS);
  if (i == 0) {
    BatchCtl* ctl = reinterpret_cast<BatchCtl*>(base + NA_CTL);
    ctl->items = items;
    ctl->nitems = nitems;
    ctl->nq = a.nq;
    for (int q = 0; q <= NQUEUE; q++) ctl->qstart[q] = a.qstart[q];
    unsigned* head = reinterpret_cast<unsigned*>(base + NA_HEAD);
    for (int q = 0; q < NQUEUE; q++) head[q * HEAD_STRIDE] = head[q * HEAD_STRIDE + 1] = 0u;
  }
  if (i >= nitems) return;
  int lo = 0, hi = a.n - 1;   // last j with start[j] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (a.start[mid] <= i) lo = mid; else hi = mid - 1;
  }
  items[i] = BatchItem{a.grid[lo], (int32_t)(i - a.start[lo])};
}

}  // namespace

// The array itself: one copy per GPU, held until the process ends.  Host code
// never passes its name to a kernel (that would be a host-side stand-in, not a
// device address); it uses the address hipGetSymbolAddress returns on each
// device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

// the device address of `scratch` on each GPU (each holds its own copy),
// looked up once per device with that device current
constexpr int NOALLOC_MAX_DEVICES = 64;
std::once_flag g_scratch_once[NOALLOC_MAX_DEVICES];
unsigned char* g_scratch_ptr[NOALLOC_MAX_DEVICES];
int g_scratch_rc[NOALLOC_MAX_DEVICES];

int scratch_of_current_device(unsigned char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return DUGKS_EDEVICE;
  if (dev >= NOALLOC_MAX_DEVICES) return DUGKS_EUNSUPPORTED;
  std::call_once(g_scratch_once[dev], [dev] {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
    g_scratch_rc[dev] = (e == hipSuccess && ptr) ? DUGKS_OK : DUGKS_EDEVICE;
  });
  *out = g_scratch_ptr[dev];
  return g_scratch_rc[dev];
}

template <typename T>
int noalloc_setup(const dugks_plan* const* plans, void* const* states, const int64_t* steps,
                  int n, int64_t nsteps, const ItemStarts& starts, unsigned char* base,
                  hipStream_t s) {
  DescChunk<T> c;
  for (int first = 0; first < n; first += DESC_CHUNK) {
    memset(&c, 0, sizeof(c));
    c.first = first;
    c.count = std::min(DESC_CHUNK, n - first);
    for (int k = 0; k < c.count; k++) {
      const dugks_plan* P = plans[first + k];
      c.d[k] = make_grid_desc<T>(P, states[first + k], P->seg_rows);
      c.st[k].n = steps[first + k];
      c.st[k].target = steps[first + k] + nsteps;
    }
    hipLaunchKernelGGL((noalloc_desc_kernel<T>), dim3(1), dim3(64), 0, s, c, base);
  }
  const int nitems = starts.start[n];
  hipLaunchKernelGGL(noalloc_items_kernel, dim3((unsigned)((nitems + 255) / 256)), dim3(256),
                     0, s, starts, base);
  return hip_status(hipGetLastError());
}

}  // namespace

extern "C" {

int dugks_step_many_noalloc(const dugks_plan* const* plans, void* const* states,
                            const int64_t* steps, int32_t n, int64_t nsteps, void* stream) {
  if (!plans || !states || !steps || n < 1 || n > NOALLOC_GRIDS || nsteps < 0)
    return DUGKS_EINVAL;
  const dugks_plan* p0 = plans[0];
  if (!p0) return DUGKS_EINVAL;
  const int precision = p0->p.precision, recon = p0->p.recon, scheme = p0->p.scheme;
  const bool mfix = (p0->p.flags & DUGKS_FLAG_MASS_FIX) != 0;
  // tiles per grid (each grid at its plan's own segment height); each grid
  // whole to one of the NQUEUE queues (one per XCD), the largest first to
  // the least loaded; within a queue the grids in decreasing order of tile
  // height, so that the short tiles fill the tail
  ItemStarts starts;
  memset(&starts, 0, sizeof(starts));
  starts.n = n;
  int order[NOALLOC_GRIDS];
  for (int j = 0; j < n; j++) {
    const dugks_plan* P = plans[j];
    if (!P || !states[j] || !aligned(states[j]) || steps[j] < 0) return DUGKS_EINVAL;
    if (P->p.precision != precision || P->p.recon != recon || P->p.scheme != scheme ||
        ((P->p.flags & DUGKS_FLAG_MASS_FIX) != 0) != mfix)
      return DUGKS_EINVAL;
    if (P->p.vel_kind == DUGKS_VEL_ARRAYS || P->p.recon == DUGKS_UPWIND5)
      return DUGKS_EUNSUPPORTED;
    order[j] = j;
  }
  // rows a grid's tiles march in all
  auto work = [plans](int j) {
    const dugks_plan* P = plans[j];
    return (int64_t)P->nstrips * ((int64_t)P->p.ny + 5 * (int64_t)P->nsegs);
  };
  std::stable_sort(order, order + n, [&](int a, int b) { return work(a) > work(b); });
  int queue_of[NOALLOC_GRIDS];
  int64_t load[NQUEUE] = {};
  for (int k = 0; k < n; k++) {
    int q = 0;
    for (int r = 1; r < NQUEUE; r++)
      if (load[r] < load[q]) q = r;
    queue_of[order[k]] = q;
    load[q] += work(order[k]);
  }
  std::stable_sort(order, order + n, [&](int a, int b) {
    if (queue_of[a] != queue_of[b]) return queue_of[a] < queue_of[b];
    return plans[a]->seg_rows > plans[b]->seg_rows;
  });
  starts.nq = NQUEUE;
  int64_t total = 0;
  int q = 0;
  for (int k = 0; k < n; k++) {
    const dugks_plan* P = plans[order[k]];
    while (q <= queue_of[order[k]]) starts.qstart[q++] = (int32_t)total;
    starts.start[k] = (int32_t)total;
    starts.grid[k] = order[k];
    total += (int64_t)P->nstrips * P->nsegs;
    if (total > NOALLOC_ITEMS) return DUGKS_EINVAL;   // beyond the array's work list
  }
  while (q <= NQUEUE) starts.qstart[q++] = (int32_t)total;
  starts.start[n] = (int32_t)total;
  if (nsteps == 0) return DUGKS_OK;
  unsigned char* base = nullptr;
  int rc = scratch_of_current_device(&base);
  if (rc) return rc;
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return DUGKS_EDEVICE;
  if ((rc = batch_occupancy(precision, recon, mfix, scheme, &per_cu)) != DUGKS_OK) return rc;
  if (per_cu < 1 || ncu < 1) return DUGKS_EDEVICE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  rc = precision == DUGKS_F64
           ? noalloc_setup<double>(plans, states, steps, n, nsteps, starts, base, s)
           : noalloc_setup<float>(plans, states, steps, n, nsteps, starts, base, s);
  if (rc) return rc;
  const BatchDev D{base + NA_DESC,
                   reinterpret_cast<SlotStep*>(base + NA_STEPS),
                   reinterpret_cast<int32_t*>(base + NA_STATUS),
                   reinterpret_cast<BatchCtl*>(base + NA_CTL),
                   reinterpret_cast<unsigned*>(base + NA_HEAD),
                   n,
                   per_cu * ncu};
  for (int64_t k = 0; k < nsteps; k++)
    if ((rc = launch_batch(D, precision, recon, mfix, scheme, s, true))) return rc;
  return DUGKS_OK;
}

}  // extern "C"
