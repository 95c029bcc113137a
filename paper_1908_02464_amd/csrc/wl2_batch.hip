// Host engine of the batched / served form (see include/weno_l2is.h):
// pooled HBM budget with first-fit sub-allocation, slot table, ragged work
// tables rebuilt on admission and retirement, and the per-step launch
// sequence captured once in a hipGraph (the kernels read the tables from
// device memory, so the graph stays valid while runs come and go; it is
// captured again only when a table outgrows its buffer or the launch shape
// changes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/weno_l2is.h"
#include "wl2_batch.hpp"
#include "wl2_desc.hpp"

using namespace wl2;

namespace {

constexpr size_t ALIGN = 256;
constexpr int ROW_BLOCKS_DEFAULT = 2048;  // persistent grid of the row kernels
constexpr int ROWS_DEFAULT = 4;           // rows per work item of a 2D run
constexpr int RED_BLOCKS = 1024;

struct SlotInfo {
  bool used = false;
  bool reported = false;
  int n[3] = {1, 1, 1};
  int dim = 1, nvar = 3;
  long long ncell = 0;
  size_t off = 0, bytes = 0;
};

size_t round_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

}  // namespace

struct weno_l2is_batch {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int max_slots = 0;
  size_t budget = 0, used = 0;
  char* pool = nullptr;
  std::vector<std::pair<size_t, size_t>> free_list;  // (offset, size), sorted
  std::vector<SlotInfo> slots;
  int active = 0;
  // device-side descriptors and tables, pinned host mirrors
  BGrid* d_grids = nullptr;
  BGrid* h_grids = nullptr;
  StepCtl* d_ctl = nullptr;
  StepCtl* h_ctl = nullptr;  // staging for admission
  RowItem* d_items[2] = {nullptr, nullptr};  // work items of the 1D / 2D runs
  RowItem* h_items[2] = {nullptr, nullptr};
  int item_cap[2] = {0, 0};
  int chunk_cap = 0;
  int* d_cslot = nullptr;
  long long* d_cfirst = nullptr;
  int* d_ccount = nullptr;
  int* h_cslot = nullptr;
  long long* h_cfirst = nullptr;
  int* h_ccount = nullptr;
  int* d_counts = nullptr;  // [0] chunks, [1] active slots, [2] 1D items, [3] 2D items
  unsigned long long* d_list = nullptr;  // cells listed for the nonlinear correction
  unsigned int* d_list_n = nullptr;
  int* h_counts = nullptr;
  int* d_slotlist = nullptr;
  int* h_slotlist = nullptr;
  SlotState* d_state = nullptr;
  SlotState* h_state = nullptr;
  int state_n = 0;
  hipEvent_t ev_state = nullptr, ev_upload = nullptr;
  bool state_pending = false, upload_pending = false;
  bool dirty = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int rows = ROWS_DEFAULT;
  int row_blocks = ROW_BLOCKS_DEFAULT;
};

namespace {

bool pool_alloc(weno_l2is_batch* b, size_t bytes, size_t* off) {
  for (size_t i = 0; i < b->free_list.size(); ++i) {
    auto& f = b->free_list[i];
    if (f.second >= bytes) {
      *off = f.first;
      f.first += bytes;
      f.second -= bytes;
      if (f.second == 0) b->free_list.erase(b->free_list.begin() + i);
      b->used += bytes;
      return true;
    }
  }
  return false;
}

void pool_free(weno_l2is_batch* b, size_t off, size_t bytes) {
  b->free_list.emplace_back(off, bytes);
  std::sort(b->free_list.begin(), b->free_list.end());
  std::vector<std::pair<size_t, size_t>> merged;
  for (auto& f : b->free_list) {
    if (!merged.empty() && merged.back().first + merged.back().second == f.first)
      merged.back().second += f.second;
    else
      merged.push_back(f);
  }
  b->free_list.swap(merged);
  b->used -= bytes;
}

// Wait until the previous table upload has been consumed before the pinned
// staging buffers are rewritten.
hipError_t wait_upload(weno_l2is_batch* b) {
  if (!b->upload_pending) return hipSuccess;
  b->upload_pending = false;
  return hipEventSynchronize(b->ev_upload);
}

void drop_graph(weno_l2is_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
}

// Item buffers of dimension index d (0: 1D, 1: 2D) for at least n items; a
// new buffer invalidates the captured graph (its kernels hold the pointer).
hipError_t reserve_items(weno_l2is_batch* b, int d, long long n) {
  if (n <= b->item_cap[d]) return hipSuccess;
  if (n > 0x3fffffffLL) return hipErrorInvalidValue;
  long long cap = b->item_cap[d] > 0 ? b->item_cap[d] : 1024;
  while (cap < n) cap *= 2;
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return e;
  b->upload_pending = false;
  RowItem *dn = nullptr, *hn = nullptr;
  if ((e = hipMalloc(&dn, sizeof(RowItem) * (size_t)cap)) != hipSuccess) return e;
  if ((e = hipHostMalloc(&hn, sizeof(RowItem) * (size_t)cap, 0)) != hipSuccess) {
    (void)hipFree(dn);
    return e;
  }
  (void)hipFree(b->d_items[d]);
  (void)hipHostFree(b->h_items[d]);
  b->d_items[d] = dn;
  b->h_items[d] = hn;
  b->item_cap[d] = (int)cap;
  drop_graph(b);
  return hipSuccess;
}

hipError_t upload_tables(weno_l2is_batch* b) {
  hipError_t e = wait_upload(b);
  if (e != hipSuccess) return e;
  // sizes first (a buffer may have to grow)
  long long need[2] = {0, 0};
  for (int s = 0; s < b->max_slots; ++s) {
    const SlotInfo& si = b->slots[s];
    if (!si.used) continue;
    const long long tiles = (si.n[0] + ROW_TILE - 1) / ROW_TILE;
    if (si.dim == 1) need[0] += tiles;
    else need[1] += tiles * ((si.n[1] + b->rows - 1) / b->rows);
  }
  for (int d = 0; d < 2; ++d)
    if ((e = reserve_items(b, d, need[d] > 0 ? need[d] : 1)) != hipSuccess) return e;
  int ni[2] = {0, 0};
  int nch = 0, nact = 0;
  for (int s = 0; s < b->max_slots; ++s) {
    const SlotInfo& si = b->slots[s];
    if (!si.used) continue;
    b->h_slotlist[nact++] = s;
    for (int x0 = 0; x0 < si.n[0]; x0 += ROW_TILE) {
      if (si.dim == 1) {
        b->h_items[0][ni[0]++] = RowItem{s, x0, 0, 1};
      } else {
        for (int y0 = 0; y0 < si.n[1]; y0 += b->rows)
          b->h_items[1][ni[1]++] = RowItem{s, x0, y0, std::min(y0 + b->rows, si.n[1])};
      }
    }
    for (long long c0 = 0; c0 < si.ncell; c0 += BATCH_CHUNK) {
      if (nch >= b->chunk_cap) return hipErrorOutOfMemory;
      b->h_cslot[nch] = s;
      b->h_cfirst[nch] = c0;
      b->h_ccount[nch] = (int)std::min<long long>(BATCH_CHUNK, si.ncell - c0);
      ++nch;
    }
  }
  b->h_counts[0] = nch;
  b->h_counts[1] = nact;
  b->h_counts[2] = ni[0];
  b->h_counts[3] = ni[1];
  hipStream_t st = b->stream;
  for (int d = 0; d < 2; ++d)
    if (ni[d] > 0 &&
        (e = hipMemcpyAsync(b->d_items[d], b->h_items[d], sizeof(RowItem) * ni[d], hipMemcpyHostToDevice, st)))
      return e;
  if ((e = hipMemcpyAsync(b->d_cslot, b->h_cslot, sizeof(int) * nch, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(b->d_cfirst, b->h_cfirst, sizeof(long long) * nch, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(b->d_ccount, b->h_ccount, sizeof(int) * nch, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(b->d_slotlist, b->h_slotlist, sizeof(int) * nact, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(b->d_counts, b->h_counts, 4 * sizeof(int), hipMemcpyHostToDevice, st)))
    return e;
  if ((e = hipEventRecord(b->ev_upload, st)) != hipSuccess) return e;
  b->upload_pending = true;
  b->state_n = nact;
  b->dirty = false;
  return hipSuccess;
}

// The launch sequence of one batched SSP-RK3 step (item buffers exist).
hipError_t enqueue_step(weno_l2is_batch* b) {
  hipStream_t st = b->stream;
  BChunks ch{0, 0, b->d_cslot, b->d_cfirst, b->d_ccount};
  hipLaunchKernelGGL(batch_cfl_kernel, dim3(RED_BLOCKS), dim3(RED_BLOCK), 0, st, b->d_grids, ch,
                     b->d_counts + 0);
  hipLaunchKernelGGL(batch_finalize_kernel, dim3(16), dim3(256), 0, st, b->d_grids, b->d_slotlist,
                     b->d_counts + 1);
  for (int stage = 0; stage < 3; ++stage) {
    hipLaunchKernelGGL(row_list_reset_kernel, dim3(1), dim3(64), 0, st, b->d_list_n);
    hipLaunchKernelGGL(batch_row_kernel<3>, dim3(b->row_blocks), dim3(RW), 0, st, b->d_grids,
                       b->d_items[0], b->d_counts + 2, stage, b->d_list, b->d_list_n);
    hipLaunchKernelGGL(batch_row_kernel<4>, dim3(b->row_blocks), dim3(RW), 0, st, b->d_grids,
                       b->d_items[1], b->d_counts + 3, stage, b->d_list, b->d_list_n);
    hipLaunchKernelGGL(batch_fix_kernel, dim3(1024), dim3(128), 0, st, b->d_grids, b->d_list,
                       b->d_list_n, stage);
  }
  return hipGetLastError();
}

hipError_t ensure_graph(weno_l2is_batch* b) {
  if (b->gexec) return hipSuccess;
  for (int d = 0; d < 2; ++d) {  // buffers exist before the capture
    hipError_t e = reserve_items(b, d, 1);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t e2 = enqueue_step(b);
  e = hipStreamEndCapture(b->stream, &b->graph);
  if (e2 != hipSuccess) return e2;
  if (e != hipSuccess) return e;
  return hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0);
}

int herr(hipError_t e) { return e == hipSuccess ? WL2_OK : WL2_E_HIP; }

}  // namespace

extern "C" {

int weno_l2is_batch_create(size_t hbm_budget_bytes, int max_slots, void* hip_stream,
                           weno_l2is_batch** out) {
  if (!out) return WL2_E_NULL;
  *out = nullptr;
  if (max_slots < 1 || max_slots > BATCH_MAX_SLOTS || hbm_budget_bytes < 4096) return WL2_E_PARAM;
  weno_l2is_batch* b = new (std::nothrow) weno_l2is_batch();
  if (!b) return WL2_E_NOMEM;
  b->stream = (hipStream_t)hip_stream;
  if (!b->stream) {
    // graph capture needs a stream other than the legacy null stream
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return WL2_E_HIP;
    }
    b->own_stream = true;
  }
  b->max_slots = max_slots;
  b->budget = hbm_budget_bytes / ALIGN * ALIGN;
  b->slots.resize(max_slots);
  // every chunk covers at least one 3-variable cell of 3 arrays (72 bytes)
  b->chunk_cap = (int)std::min<size_t>((size_t)1 << 26, b->budget / (72 * BATCH_CHUNK) + max_slots + 16);
  // a list entry per admissible cell (at least 72 bytes of state each)
  const size_t list_cap = b->budget / 72 + 1;
  bool ok = hipMalloc(&b->pool, b->budget) == hipSuccess &&
            hipMalloc(&b->d_list, sizeof(unsigned long long) * list_cap) == hipSuccess &&
            hipMalloc(&b->d_list_n, sizeof(unsigned int)) == hipSuccess &&
            hipMalloc(&b->d_grids, sizeof(BGrid) * max_slots) == hipSuccess &&
            hipMalloc(&b->d_ctl, sizeof(StepCtl) * max_slots) == hipSuccess &&
            hipMalloc(&b->d_cslot, sizeof(int) * b->chunk_cap) == hipSuccess &&
            hipMalloc(&b->d_cfirst, sizeof(long long) * b->chunk_cap) == hipSuccess &&
            hipMalloc(&b->d_ccount, sizeof(int) * b->chunk_cap) == hipSuccess &&
            hipMalloc(&b->d_counts, 4 * sizeof(int)) == hipSuccess &&
            hipMalloc(&b->d_slotlist, sizeof(int) * max_slots) == hipSuccess &&
            hipMalloc(&b->d_state, sizeof(SlotState) * max_slots) == hipSuccess &&
            hipHostMalloc(&b->h_grids, sizeof(BGrid) * max_slots, 0) == hipSuccess &&
            hipHostMalloc(&b->h_ctl, sizeof(StepCtl) * max_slots, 0) == hipSuccess &&
            hipHostMalloc(&b->h_cslot, sizeof(int) * b->chunk_cap, 0) == hipSuccess &&
            hipHostMalloc(&b->h_cfirst, sizeof(long long) * b->chunk_cap, 0) == hipSuccess &&
            hipHostMalloc(&b->h_ccount, sizeof(int) * b->chunk_cap, 0) == hipSuccess &&
            hipHostMalloc(&b->h_counts, 4 * sizeof(int), 0) == hipSuccess &&
            hipHostMalloc(&b->h_slotlist, sizeof(int) * max_slots, 0) == hipSuccess &&
            hipHostMalloc(&b->h_state, sizeof(SlotState) * max_slots, 0) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev_state, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev_upload, hipEventDisableTiming) == hipSuccess;
  if (ok) {
    b->free_list.emplace_back(0, b->budget);
    std::memset(b->h_counts, 0, 4 * sizeof(int));
    std::memset(b->h_grids, 0, sizeof(BGrid) * max_slots);
    ok = hipMemcpyAsync(b->d_grids, b->h_grids, sizeof(BGrid) * max_slots, hipMemcpyHostToDevice,
                        b->stream) == hipSuccess &&
         hipMemcpyAsync(b->d_counts, b->h_counts, 4 * sizeof(int), hipMemcpyHostToDevice,
                        b->stream) == hipSuccess &&
         hipStreamSynchronize(b->stream) == hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();
    weno_l2is_batch_destroy(b);
    return WL2_E_NOMEM;
  }
  *out = b;
  return WL2_OK;
}

int weno_l2is_batch_admit(weno_l2is_batch* b, int nx, int ny, int nz, double dx, double gamma,
                          const weno_l2is_params* p, const double* U0, int u0_on_host,
                          double t_end, int* slot, size_t* bytes_out) {
  if (!b || !p || !U0 || !slot) return WL2_E_NULL;
  int rc = validate_grid(nx, ny, nz, dx, gamma, p);
  if (rc) return rc;
  if (nz > 1) return WL2_E_SHAPE;
  if (p->split == WL2_SPLIT_LF) return WL2_E_PARAM;
  if (p->bc[0] == WL2_BC_INFLOW) return WL2_E_BC;
  if (p->bc[2] >= WL2_BC_STATE_WALL || p->bc[3] >= WL2_BC_STATE_WALL) return WL2_E_BC;
  if (!(t_end > 0.0) || !(t_end < 1e300)) return WL2_E_PARAM;
  int s = -1;
  for (int i = 0; i < b->max_slots; ++i)
    if (!b->slots[i].used) {
      s = i;
      break;
    }
  if (s < 0) return WL2_E_BUDGET;
  SlotInfo si;
  si.n[0] = nx;
  si.n[1] = ny;
  si.n[2] = 1;
  si.dim = grid_dim(ny, nz);
  si.nvar = si.dim + 2;
  si.ncell = (long long)nx * ny;
  const size_t arr = round_up(sizeof(double) * (size_t)si.nvar * si.ncell);
  si.bytes = arr * 3;
  if (!pool_alloc(b, si.bytes, &si.off)) return WL2_E_BUDGET;
  hipError_t e = wait_upload(b);
  if (e != hipSuccess) {
    pool_free(b, si.off, si.bytes);
    return WL2_E_HIP;
  }
  BGrid& G = b->h_grids[s];
  std::memset(&G, 0, sizeof(G));
  fill_grid_desc(si.n, si.dim, dx, gamma, *p, G.g, G.ph);
  char* base = b->pool + si.off;
  G.U = (double*)base;
  G.U1 = (double*)(base + arr);
  G.U2 = (double*)(base + 2 * arr);
  G.ctl = b->d_ctl + s;
  G.cfl_dx = p->cfl * dx;
  G.dim = si.dim;
  G.nv = si.nvar;
  G.active = 1;
  StepCtl& C = b->h_ctl[s];
  std::memset(&C, 0, sizeof(C));
  C.t = 0.0;
  C.t_end = t_end;
  const size_t ubytes = sizeof(double) * (size_t)si.nvar * si.ncell;
  hipStream_t st = b->stream;
  if ((e = hipMemcpyAsync(G.U, U0, ubytes, u0_on_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st)) ||
      (e = hipMemcpyAsync(b->d_grids + s, &G, sizeof(BGrid), hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(b->d_ctl + s, &C, sizeof(StepCtl), hipMemcpyHostToDevice, st)) ||
      (e = hipEventRecord(b->ev_upload, st))) {
    pool_free(b, si.off, si.bytes);
    return WL2_E_HIP;
  }
  b->upload_pending = true;  // h_grids[s] / h_ctl[s] are in flight
  if (u0_on_host) {
    // a pageable host source must not change before the copy has run
    if (hipStreamSynchronize(st) != hipSuccess) return WL2_E_HIP;
    b->upload_pending = false;
  }
  si.used = true;
  si.reported = false;
  b->slots[s] = si;
  b->active++;
  b->dirty = true;
  b->state_pending = false;  // snapshots before this admission are stale
  *slot = s;
  if (bytes_out) *bytes_out = si.bytes;
  return WL2_OK;
}

int weno_l2is_batch_advance(weno_l2is_batch* b, int n_steps) {
  if (!b) return WL2_E_NULL;
  if (n_steps < 0) return WL2_E_PARAM;
  hipError_t e;
  if (b->dirty && (e = upload_tables(b)) != hipSuccess) return herr(e);
  if (b->active == 0) return WL2_OK;
  if ((e = ensure_graph(b)) != hipSuccess) return herr(e);
  for (int k = 0; k < n_steps; ++k)
    if ((e = hipGraphLaunch(b->gexec, b->stream)) != hipSuccess) return herr(e);
  hipLaunchKernelGGL(batch_gather_kernel, dim3(4), dim3(256), 0, b->stream, b->d_grids,
                     b->d_slotlist, b->d_counts + 1, b->d_state);
  if ((e = hipGetLastError()) != hipSuccess) return herr(e);
  if ((e = hipMemcpyAsync(b->h_state, b->d_state, sizeof(SlotState) * b->state_n,
                          hipMemcpyDeviceToHost, b->stream)) != hipSuccess)
    return herr(e);
  if ((e = hipEventRecord(b->ev_state, b->stream)) != hipSuccess) return herr(e);
  b->state_pending = true;
  return WL2_OK;
}

int weno_l2is_batch_poll(weno_l2is_batch* b, int* done_slots, int cap, int* n_done) {
  if (!b || !n_done || (cap > 0 && !done_slots)) return WL2_E_NULL;
  *n_done = 0;
  if (!b->state_pending) return WL2_OK;
  const hipError_t q = hipEventQuery(b->ev_state);
  if (q == hipErrorNotReady) return WL2_OK;
  if (q != hipSuccess) return WL2_E_HIP;
  int k = 0;
  for (int i = 0; i < b->state_n && k < cap; ++i) {
    const SlotState& ss = b->h_state[i];
    if (ss.slot < 0 || ss.slot >= b->max_slots) continue;
    SlotInfo& si = b->slots[ss.slot];
    if (!si.used || si.reported) continue;
    if (!(ss.t < ss.t_end) || ss.status != 0u) {
      si.reported = true;
      done_slots[k++] = ss.slot;
    }
  }
  *n_done = k;
  return WL2_OK;
}

int weno_l2is_batch_fetch(weno_l2is_batch* b, int slot, double* U_out, int out_on_host,
                          double* t_out, unsigned* status, unsigned* steps) {
  if (!b || !U_out) return WL2_E_NULL;
  if (slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return WL2_E_SLOT;
  SlotInfo& si = b->slots[slot];
  const BGrid& G = b->h_grids[slot];
  StepCtl C;
  const size_t ubytes = sizeof(double) * (size_t)si.nvar * si.ncell;
  hipError_t e;
  if ((e = hipMemcpyAsync(U_out, G.U, ubytes, out_on_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                          b->stream)) ||
      (e = hipMemcpyAsync(&C, b->d_ctl + slot, sizeof(C), hipMemcpyDeviceToHost, b->stream)) ||
      (e = hipStreamSynchronize(b->stream)))
    return herr(e);
  b->upload_pending = false;
  if (t_out) *t_out = C.t;
  if (status) *status = C.status;
  if (steps) *steps = C.steps;
  pool_free(b, si.off, si.bytes);
  si.used = false;
  b->h_grids[slot].active = 0;
  b->active--;
  b->dirty = true;
  b->state_pending = false;  // snapshots before this retirement are stale
  return WL2_OK;
}

int weno_l2is_batch_tune(weno_l2is_batch* b, int rows, int blocks) {
  if (!b) return WL2_E_NULL;
  if (rows < 0 || rows > ROW_MAX_YCH) return WL2_E_PARAM;
  if (blocks != 0 && (blocks < 64 || blocks > 65536)) return WL2_E_PARAM;
  if (rows && rows != b->rows) {
    b->rows = rows;
    b->dirty = true;  // the 2D items follow the rows per item
  }
  if (blocks && blocks != b->row_blocks) {
    b->row_blocks = blocks;
    drop_graph(b);  // the grid size is part of the captured launches
  }
  return WL2_OK;
}

int weno_l2is_batch_usage(weno_l2is_batch* b, size_t* used_bytes, int* active) {
  if (!b) return WL2_E_NULL;
  if (used_bytes) *used_bytes = b->used;
  if (active) *active = b->active;
  return WL2_OK;
}

void weno_l2is_batch_destroy(weno_l2is_batch* b) {
  if (!b) return;
  if (b->stream || b->pool) (void)hipStreamSynchronize(b->stream);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->ev_state) (void)hipEventDestroy(b->ev_state);
  if (b->ev_upload) (void)hipEventDestroy(b->ev_upload);
  (void)hipFree(b->pool);
  (void)hipFree(b->d_list);
  (void)hipFree(b->d_list_n);
  (void)hipFree(b->d_grids);
  (void)hipFree(b->d_ctl);
  for (int d = 0; d < 2; ++d) {
    (void)hipFree(b->d_items[d]);
    (void)hipHostFree(b->h_items[d]);
  }
  (void)hipFree(b->d_cslot);
  (void)hipFree(b->d_cfirst);
  (void)hipFree(b->d_ccount);
  (void)hipFree(b->d_counts);
  (void)hipFree(b->d_slotlist);
  (void)hipFree(b->d_state);
  (void)hipHostFree(b->h_grids);
  (void)hipHostFree(b->h_ctl);
  (void)hipHostFree(b->h_cslot);
  (void)hipHostFree(b->h_cfirst);
  (void)hipHostFree(b->h_ccount);
  (void)hipHostFree(b->h_counts);
  (void)hipHostFree(b->h_slotlist);
  (void)hipHostFree(b->h_state);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"
