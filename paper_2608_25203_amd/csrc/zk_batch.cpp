// zk_batch.cpp -- many independent tiles of uneven sizes and orders stepped
// together (C ABI in zk.h).
//
// Each tile keeps its own context (plan, tables, spectra) in a slice of the
// batch workspace.  The tiles' launch sequences are merged into phases: a
// phase takes the next launch of every tile whose next launch is a row pass
// (or, alternately, a column pass), choosing the kind the tile with the most
// launches left needs.  Within a phase, tiles of one size share one batched
// launch: blockIdx.y runs over (tile, program or task) items, each reading
// its tile's argument record from a device table.  The phases of one RK4
// step are recorded once as a HIP graph (kernel nodes only) and replayed;
// or (ZK_BATCH_OPT_PERSISTENT) each merged segment runs as one persistent
// launch whose workers take (tile, pass, item, block chunk) units in phase
// order and wait on per-tile completion counters (zk_persist.hpp).
// The team shape (T threads, radix E) of each pass and size is chosen by an
// empirical autotuner among the compiled shapes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "zk.h"
#include "zk_ctx_internal.hpp"
#include "zk_kernels.hpp"
#include "zk_persist.hpp"

using namespace zk;

namespace {

struct BL {  // one batched launch
  bool row, pad;
  int nx, ny;
  int T, E, blocks;
  int item0, nitems;
};
using Phase = std::vector<BL>;
using Key = std::tuple<int, int, int, int>;  // row, pad, nx, ny

constexpr int kSegs = 7;  // entry, body0+lift1, body1+lift0, body0, body1, exit0, exit1

}  // namespace

struct zk_batch {
  std::vector<zk_ctx *> tiles;
  std::vector<size_t> off;
  double g = 9.81;
  int precision = 32;
  size_t off_rargs = 0, off_cargs = 0, off_items = 0, items_cap = 0, total = 0;
  char *ws = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;
  bool bound = false;
  std::vector<double *> eta, psi;
  bool have_fields = false;
  double dt = NAN;
  bool ready = false;
  bool use_graph = true;
  std::map<Key, std::pair<int, int>> tune;
  std::vector<Phase> seg[kSegs];
  std::vector<BatchItem> items;
  hipGraphExec_t exec[kSegs] = {};
  // persistent form
  bool persistent = false;
  size_t off_units = 0, units_cap = 0, off_ctr = 0;
  std::vector<PUnit> units;
  size_t useg0[kSegs] = {}, usegn[kSegs] = {};
  int useg_lds[kSegs] = {};
  int workers = 0;
  uint32_t spin_limit = 1u << 20;  // sleeps of ~0.1 us each: a wait gives up after about 0.1-1 s
  std::string err;
  long long launches_per_step = 0, phases_per_step = 0;
  ~zk_batch() {
    for (auto &e : exec)
      if (e) hipGraphExecDestroy(e);
    for (auto *c : tiles) zk_destroy(c);
  }
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int fail(zk_batch *b, int code, const std::string &m) {
  if (b) b->err = m;
  return code;
}
int hip_fail(zk_batch *b, hipError_t e, const char *what) {
  return fail(b, ZK_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIP_TRY(b, call)                                 \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(b, e_, #call); \
  } while (0)

bool is_row(int kind) { return kind == L_ROW_PAD || kind == L_ROW_BASE; }

const void *kernel_for(const zk_batch *b, bool row, int T, int E, bool pad) {
  if (b->precision == 32) return row ? batch_row_kernel<float>(T, E, pad) : batch_col_kernel<float>(T, E, pad);
  return row ? batch_row_kernel<double>(T, E, pad) : batch_col_kernel<double>(T, E, pad);
}

// Candidate team shapes of a transform of an axis of n points (radix_candidates),
// T in {16, ..., 1024} threads.
std::vector<std::pair<int, int>> candidates(const zk_batch *b, bool row, bool pad, int n) {
  std::vector<std::pair<int, int>> out;
  const int N = pad ? 3 * n / 2 : n;
  int cand[3];
  const int ncand = radix_candidates(n, pad, cand);
  for (int ci = 0; ci < ncand; ++ci) {
    const int E = cand[ci];
    if (N % E) continue;
    const int T = N / E;
    if (b->persistent && persist_shape(row, T, E) < 0) continue;  // not hosted by the persistent kernel
    if (T >= 2 && T <= 1024 && !(T & (T - 1)) && kernel_for(b, row, T, E, pad)) out.push_back({T, E});
  }
  return out;
}

std::pair<int, int> shape_of(zk_batch *b, bool row, bool pad, int nx, int ny) {
  const Key k{row, pad, nx, ny};
  auto it = b->tune.find(k);
  if (it != b->tune.end()) return it->second;
  const int n = row ? nx : ny;  // default: the smallest first-pass radix (as a single context)
  const int E = default_radix(n, pad);
  return {(pad ? 3 * n / 2 : n) / E, E};
}

int blocks_of(bool row, bool pad, int nx, int ny, int T) {
  const int per = T < 256 ? 256 / T : 1;  // teams per block; a partial last block idles its spare teams
  return row ? ((pad ? 3 * ny / 2 : ny) + per - 1) / per : (nx / 2 + per - 1) / per;
}

// Merge the tiles' sequences of one segment into phases and append items.
void merge(zk_batch *b, const std::vector<std::vector<Launch>> &seqs, std::vector<Phase> &out) {
  const int nt = (int)seqs.size();
  std::vector<size_t> pos(nt, 0);
  for (;;) {
    int best = -1;
    size_t left = 0;
    for (int t = 0; t < nt; ++t)
      if (seqs[t].size() - pos[t] > left) {
        left = seqs[t].size() - pos[t];
        best = t;
      }
    if (best < 0) break;
    const bool row = is_row(seqs[best][pos[best]].kind);
    std::map<Key, std::vector<std::pair<int, const Launch *>>> groups;
    for (int t = 0; t < nt; ++t) {
      if (pos[t] >= seqs[t].size()) continue;
      const Launch &l = seqs[t][pos[t]];
      if (is_row(l.kind) != row) continue;
      const zk_ctx *c = b->tiles[t];
      const bool pad = l.kind == L_ROW_PAD || l.kind == L_COL_PAD;
      groups[Key{row, pad, c->pp.nx, c->pp.ny}].push_back({t, &l});
      ++pos[t];
    }
    Phase ph;
    for (auto &kv : groups) {
      const bool pad = std::get<1>(kv.first);
      const int nx = std::get<2>(kv.first), ny = std::get<3>(kv.first);
      const auto sh = shape_of(b, row, pad, nx, ny);
      BL bl{row, pad, nx, ny, sh.first, sh.second, blocks_of(row, pad, nx, ny, sh.first), (int)b->items.size(), 0};
      for (auto &tl : kv.second)
        for (int k = tl.second->first; k < tl.second->first + tl.second->count; ++k)
          b->items.push_back(BatchItem{2 * tl.first + (pad ? 0 : 1), k});
      bl.nitems = (int)b->items.size() - bl.item0;
      ph.push_back(bl);
    }
    // larger tiles first: their blocks start early
    std::sort(ph.begin(), ph.end(), [](const BL &x, const BL &y) { return x.nx * x.ny > y.nx * y.ny; });
    out.push_back(std::move(ph));
  }
}

void kernel_params(const zk_batch *b, const BL &l, const void **fn, void **args_dev, BatchItem **items_dev) {
  *fn = kernel_for(b, l.row, l.T, l.E, l.pad);
  *args_dev = b->ws + (l.row ? b->off_rargs : b->off_cargs);
  *items_dev = reinterpret_cast<BatchItem *>(b->ws + b->off_items) + l.item0;
}

int launch(zk_batch *b, const BL &l) {
  const void *fn;
  void *args;
  BatchItem *it;
  kernel_params(b, l, &fn, &args, &it);
  if (!fn) return fail(b, ZK_EINVAL, "team shape not built");
  PhysArgs ph{};
  int tile0 = 0, first0 = 0;  // unused: batches pass their item table
  const void *sched0 = nullptr;  // and read each tile's schedule from its record
  void *params[] = {&args, &it, &tile0, &first0, &sched0, &ph};
  HIP_TRY(b, hipLaunchKernel(fn, dim3(l.blocks, l.nitems), dim3(std::max(256, l.T)), params, 0, b->stream));
  return ZK_OK;
}

int build_graph(zk_batch *b, int s) {
  if (b->exec[s]) {
    HIP_TRY(b, hipGraphExecDestroy(b->exec[s]));
    b->exec[s] = nullptr;
  }
  hipGraph_t g;
  HIP_TRY(b, hipGraphCreate(&g, 0));
  std::vector<hipGraphNode_t> prev, cur;
  int rc = ZK_OK;
  for (const Phase &ph : b->seg[s]) {
    cur.clear();
    for (const BL &l : ph) {
      const void *fn;
      void *args;
      BatchItem *it;
      kernel_params(b, l, &fn, &args, &it);
      if (!fn) {
        rc = fail(b, ZK_EINVAL, "team shape not built");
        break;
      }
      PhysArgs ph{};
      int tile0 = 0, first0 = 0;  // unused: batches pass their item table
      const void *sched0 = nullptr;  // and read each tile's schedule from its record
      void *params[] = {&args, &it, &tile0, &first0, &sched0, &ph};
      hipKernelNodeParams p{};
      p.func = const_cast<void *>(fn);
      p.gridDim = dim3(l.blocks, l.nitems);
      p.blockDim = dim3(std::max(256, l.T));
      p.sharedMemBytes = 0;
      p.kernelParams = params;
      p.extra = nullptr;
      hipGraphNode_t node;
      const hipError_t e = hipGraphAddKernelNode(&node, g, prev.empty() ? nullptr : prev.data(), prev.size(), &p);
      if (e != hipSuccess) {
        rc = hip_fail(b, e, "hipGraphAddKernelNode");
        break;
      }
      cur.push_back(node);
    }
    if (rc) break;
    prev.swap(cur);
  }
  if (!rc) {
    const hipError_t e = hipGraphInstantiate(&b->exec[s], g, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = hip_fail(b, e, "hipGraphInstantiate");
  }
  hipGraphDestroy(g);
  return rc;
}

// Blocks of kPBlock threads (kPBlock / T teams each) covering a pass.
int pblocks_of(bool row, bool pad, int nx, int ny, int T) {
  const int per = kPBlock / T;
  return row ? ((pad ? 3 * ny / 2 : ny) + per - 1) / per : (nx / 2 + per - 1) / per;
}

// Units of the persistent form, segment by segment, in phase order: each
// item of each batched launch is cut into at most kUnitsPerItem chunks of at
// least kMinUnitBlocks consecutive blocks; a unit waits for every unit of
// its tile's earlier phases in the same segment.
constexpr int kUnitsPerItem = 32, kMinUnitBlocks = 2, kStagger = 8;
int build_units(zk_batch *b) {
  const int nt = (int)b->tiles.size();
  b->units.clear();
  int maxlds = 0;
  std::vector<uint32_t> cum(nt), start(nt);
  for (int s = 0; s < kSegs; ++s) {
    b->useg0[s] = b->units.size();
    b->useg_lds[s] = 0;
    std::fill(cum.begin(), cum.end(), 0u);
    std::vector<int> key;  // queue position: the phase, staggered by tile
    int pi = 0;
    for (const Phase &ph : b->seg[s]) {
      start = cum;
      for (const BL &l : ph) {
        const int shape = persist_shape(l.row, l.T, l.E);
        if (shape < 0)
          return fail(b, ZK_EINVAL, "persistent form: the tiles' axes must be powers of two whose transforms "
                                    "are 128 to 1024 points, with the smallest first-pass radix");
        const int lds = b->precision == 32 ? persist_lds_bytes<float>(shape) : persist_lds_bytes<double>(shape);
        b->useg_lds[s] = std::max(b->useg_lds[s], lds);
        const int nblk = pblocks_of(l.row, l.pad, l.nx, l.ny, l.T);
        const int chunk = std::max(kMinUnitBlocks, (nblk + kUnitsPerItem - 1) / kUnitsPerItem);
        for (int k = l.item0; k < l.item0 + l.nitems; ++k) {
          const BatchItem it = b->items[k];
          const int t = it.tile / 2;
          for (int b0 = 0; b0 < nblk; b0 += chunk) {
            b->units.push_back(PUnit{shape, it.tile, it.index, b0, std::min(chunk, nblk - b0), t, start[t], 0});
            key.push_back(pi + t % kStagger);
            ++cum[t];
          }
        }
      }
      ++pi;
    }
    // Tile t's phase p is queued at slot p + (t mod kStagger): a tile's next
    // phase never follows its current one directly, while each tile's phases
    // (all a unit waits on) stay in order, earlier in the queue.
    {
      const size_t u0 = b->useg0[s], nu = b->units.size() - u0;
      std::vector<size_t> ord(nu);
      for (size_t i = 0; i < nu; ++i) ord[i] = i;
      std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return key[x] < key[y]; });
      std::vector<PUnit> seg(nu);
      for (size_t i = 0; i < nu; ++i) seg[i] = b->units[u0 + ord[i]];
      std::copy(seg.begin(), seg.end(), b->units.begin() + u0);
    }
    b->usegn[s] = b->units.size() - b->useg0[s];
    maxlds = std::max(maxlds, b->useg_lds[s]);
  }
  if (b->units.size() > b->units_cap) return fail(b, ZK_EINVAL, "persistent schedule exceeds its reserved capacity");
  int cus = 0;
  HIP_TRY(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
  const int per = b->precision == 32 ? persistent_blocks_per_cu<float>(maxlds) : persistent_blocks_per_cu<double>(maxlds);
  if (per < 1 || cus < 1) return fail(b, ZK_EDEVICE, "persistent kernel does not fit a compute unit");
  b->workers = per * cus;
  return ZK_OK;
}

// Plans for dt, argument tables, merged schedules and graphs.
int prepare(zk_batch *b, double dt) {
  if (b->ready && dt == b->dt) return ZK_OK;
  const int nt = (int)b->tiles.size();
  for (auto *c : b->tiles) {
    const int rc = ctx_upload(c, dt);
    if (rc) return fail(b, rc, std::string("tile plan: ") + zk_last_error(c));
  }
  // argument tables: [2 t + (pad ? 0 : 1)]
  const size_t rsz = b->precision == 32 ? sizeof(RowArgs<float>) : sizeof(RowArgs<double>);
  const size_t csz = b->precision == 32 ? sizeof(ColArgs<float>) : sizeof(ColArgs<double>);
  std::vector<char> rtab(2 * nt * rsz), ctab(2 * nt * csz);
  for (int t = 0; t < nt; ++t) {
    Phys ph;
    ph.in0 = b->eta[t];
    ph.in1 = b->psi[t];
    ph.out0 = b->eta[t];
    ph.out1 = b->psi[t];
    for (int p = 0; p < 2; ++p) {
      const bool pad = p == 0;
      if (b->precision == 32) {
        const RowArgs<float> r = ctx_row_args<float>(b->tiles[t], pad, ph, 0);
        const ColArgs<float> c = ctx_col_args<float>(b->tiles[t], pad, 0);
        std::memcpy(&rtab[(2 * t + p) * rsz], &r, rsz);
        std::memcpy(&ctab[(2 * t + p) * csz], &c, csz);
      } else {
        const RowArgs<double> r = ctx_row_args<double>(b->tiles[t], pad, ph, 0);
        const ColArgs<double> c = ctx_col_args<double>(b->tiles[t], pad, 0);
        std::memcpy(&rtab[(2 * t + p) * rsz], &r, rsz);
        std::memcpy(&ctab[(2 * t + p) * csz], &c, csz);
      }
    }
  }
  // merged schedules
  b->items.clear();
  std::vector<std::vector<Launch>> seqs(nt);
  auto build = [&](int s, auto pick) {
    for (int t = 0; t < nt; ++t) seqs[t] = pick(b->tiles[t]->plan);
    b->seg[s].clear();
    merge(b, seqs, b->seg[s]);
  };
  auto cat = [](const std::vector<Launch> &x, const std::vector<Launch> &y) {
    std::vector<Launch> r(x);
    r.insert(r.end(), y.begin(), y.end());
    return r;
  };
  build(0, [](const Plan &p) { return p.step_entry; });
  build(1, [&](const Plan &p) { return cat(p.step_body[0], p.step_lift[1]); });
  build(2, [&](const Plan &p) { return cat(p.step_body[1], p.step_lift[0]); });
  build(3, [](const Plan &p) { return p.step_body[0]; });
  build(4, [](const Plan &p) { return p.step_body[1]; });
  build(5, [](const Plan &p) { return p.step_exit[0]; });
  build(6, [](const Plan &p) { return p.step_exit[1]; });
  if (b->items.size() > b->items_cap) return fail(b, ZK_EINVAL, "batched schedule exceeds its reserved capacity");
  b->phases_per_step = (long long)b->seg[1].size();
  b->launches_per_step = 0;
  for (auto &ph : b->seg[1]) b->launches_per_step += (long long)ph.size();
  if (b->persistent) {
    const int rc = build_units(b);
    if (rc) return rc;
    b->launches_per_step = 1;
  }
  HIP_TRY(b, hipSetDevice(b->device));
  HIP_TRY(b, hipMemcpyAsync(b->ws + b->off_rargs, rtab.data(), rtab.size(), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(b, hipMemcpyAsync(b->ws + b->off_cargs, ctab.data(), ctab.size(), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(b, hipMemcpyAsync(b->ws + b->off_items, b->items.data(), b->items.size() * sizeof(BatchItem),
                            hipMemcpyHostToDevice, b->stream));
  if (b->persistent && !b->units.empty())
    HIP_TRY(b, hipMemcpyAsync(b->ws + b->off_units, b->units.data(), b->units.size() * sizeof(PUnit),
                              hipMemcpyHostToDevice, b->stream));
  HIP_TRY(b, hipStreamSynchronize(b->stream));
  if (b->use_graph && !b->persistent)
    for (int s = 0; s < kSegs; ++s) {
      const int rc = build_graph(b, s);
      if (rc) return rc;
    }
  b->dt = dt;
  b->ready = true;
  return ZK_OK;
}

int run_seg(zk_batch *b, int s) {
  if (b->persistent) {
    if (!b->usegn[s]) return ZK_OK;
    uint32_t *ctr = reinterpret_cast<uint32_t *>(b->ws + b->off_ctr);
    const PUnit *u = reinterpret_cast<const PUnit *>(b->ws + b->off_units) + b->useg0[s];
    HIP_TRY(b, launch_persist_reset(ctr, (int)b->tiles.size(), b->stream));
    if (b->precision == 32)
      HIP_TRY(b, launch_persistent<float>(b->workers, b->useg_lds[s], b->stream,
                                          reinterpret_cast<const RowArgs<float> *>(b->ws + b->off_rargs),
                                          reinterpret_cast<const ColArgs<float> *>(b->ws + b->off_cargs), u,
                                          (int)b->usegn[s], ctr, b->spin_limit));
    else
      HIP_TRY(b, launch_persistent<double>(b->workers, b->useg_lds[s], b->stream,
                                           reinterpret_cast<const RowArgs<double> *>(b->ws + b->off_rargs),
                                           reinterpret_cast<const ColArgs<double> *>(b->ws + b->off_cargs), u,
                                           (int)b->usegn[s], ctr, b->spin_limit));
    return ZK_OK;
  }
  if (b->use_graph) {
    HIP_TRY(b, hipGraphLaunch(b->exec[s], b->stream));
    return ZK_OK;
  }
  for (const Phase &ph : b->seg[s])
    for (const BL &l : ph) {
      const int rc = launch(b, l);
      if (rc) return rc;
    }
  return ZK_OK;
}

int check(zk_batch *b) {
  if (!b) return ZK_EINVAL;
  b->err.clear();
  if (!b->bound) return fail(b, ZK_ENOWS, "workspace not bound (call zk_batch_bind)");
  if (!b->have_fields) return fail(b, ZK_EINVAL, "fields not set (call zk_batch_set_fields)");
  HIP_TRY(b, hipSetDevice(b->device));
  return ZK_OK;
}

}  // namespace

extern "C" {

zk_batch *zk_batch_create(int ntiles, const zk_tile *tiles, double g, int precision) {
  if (ntiles < 1 || ntiles > 4096 || !tiles || !(g > 0) || (precision != 32 && precision != 64)) return nullptr;
  zk_batch *b = new (std::nothrow) zk_batch();
  if (!b) return nullptr;
  b->g = g;
  b->precision = precision;
  size_t off = 0, items = 0;
  for (int t = 0; t < ntiles; ++t) {
    const zk_tile &d = tiles[t];
    if (d.ny == 1) {  // 1D grids run as single contexts only
      delete b;
      return nullptr;
    }
    zk_ctx *c = zk_create(d.nx, d.ny, d.Lx, d.Ly, d.depth, g, d.M);
    if (!c || zk_set_option(c, ZK_OPT_PRECISION, precision) || zk_set_option(c, ZK_OPT_CHECK, 0)) {
      if (c) zk_destroy(c);
      delete b;
      return nullptr;
    }
    b->tiles.push_back(c);
    b->off.push_back(off);
    off = align_up(off + zk_workspace_bytes(c));
    // items: every program or task of every launch of a step's segments
    const Plan probe = build_plan(c->pp, 1.0);
    auto count = [&](const std::vector<Launch> &s) {
      for (const Launch &l : s) items += (size_t)std::max(0, l.count);
    };
    for (auto *s : {&probe.step_entry, &probe.step_body[0], &probe.step_body[1], &probe.step_lift[0],
                    &probe.step_lift[1], &probe.step_exit[0], &probe.step_exit[1]})
      count(*s);
    count(probe.step_body[0]);  // body segments appear twice (with and without the lift)
    count(probe.step_body[1]);
  }
  const size_t rsz = precision == 32 ? sizeof(RowArgs<float>) : sizeof(RowArgs<double>);
  const size_t csz = precision == 32 ? sizeof(ColArgs<float>) : sizeof(ColArgs<double>);
  b->off_rargs = off;
  off = align_up(off + 2 * ntiles * rsz);
  b->off_cargs = off;
  off = align_up(off + 2 * ntiles * csz);
  b->items_cap = items;
  b->off_items = off;
  off = align_up(off + items * sizeof(BatchItem));
  b->units_cap = items * kUnitsPerItem;
  b->off_units = off;
  off = align_up(off + b->units_cap * sizeof(PUnit));
  b->off_ctr = off;
  off = align_up(off + (size_t)(kCtrDone + ntiles) * sizeof(uint32_t));
  b->total = off;
  b->eta.assign(ntiles, nullptr);
  b->psi.assign(ntiles, nullptr);
  return b;
}

void zk_batch_destroy(zk_batch *b) { delete b; }

size_t zk_batch_workspace_bytes(const zk_batch *b) { return b ? b->total : 0; }

int zk_batch_bind(zk_batch *b, void *ws, size_t bytes, void *stream) {
  if (!b) return ZK_EINVAL;
  b->err.clear();
  if (!ws || ((uintptr_t)ws % kAlign) != 0) return fail(b, ZK_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < b->total) return fail(b, ZK_ENOWS, "workspace smaller than zk_batch_workspace_bytes");
  HIP_TRY(b, hipGetDevice(&b->device));
  b->ws = static_cast<char *>(ws);
  b->stream = static_cast<hipStream_t>(stream);
  for (size_t t = 0; t < b->tiles.size(); ++t) {
    const int rc = zk_bind(b->tiles[t], b->ws + b->off[t], zk_workspace_bytes(b->tiles[t]), stream);
    if (rc) return fail(b, rc, std::string("tile bind: ") + zk_last_error(b->tiles[t]));
  }
  b->bound = true;
  b->ready = false;
  return ZK_OK;
}

int zk_batch_set_fields(zk_batch *b, double *const *eta, double *const *psi) {
  if (!b) return ZK_EINVAL;
  b->err.clear();
  if (!eta || !psi) return fail(b, ZK_EINVAL, "null field arrays");
  for (size_t t = 0; t < b->tiles.size(); ++t) {
    if (!eta[t] || !psi[t] || ((uintptr_t)eta[t] & 15u) || ((uintptr_t)psi[t] & 15u))
      return fail(b, ZK_EINVAL, "null or misaligned tile field");
    b->eta[t] = eta[t];
    b->psi[t] = psi[t];
  }
  b->have_fields = true;
  b->ready = false;
  return ZK_OK;
}

int zk_batch_set_option(zk_batch *b, int key, double value) {
  if (!b) return ZK_EINVAL;
  b->err.clear();
  if (key == ZK_BATCH_OPT_GRAPH) {
    b->use_graph = value != 0.0;
    b->ready = false;
    return ZK_OK;
  }
  if (key == ZK_BATCH_OPT_PERSISTENT) {
    b->persistent = value != 0.0;
    b->tune.clear();  // shapes are re-chosen among those the form hosts
    b->ready = false;
    return ZK_OK;
  }
  return fail(b, ZK_EINVAL, "unknown batch option");
}

int zk_batch_step(zk_batch *b, double dt, int nsteps) {
  int rc = check(b);
  if (rc) return rc;
  if (!std::isfinite(dt) || nsteps < 0) return fail(b, ZK_EINVAL, "dt must be finite and nsteps >= 0");
  if (nsteps == 0) return ZK_OK;
  if ((rc = prepare(b, dt))) return rc;
  uint32_t *ctr = reinterpret_cast<uint32_t *>(b->ws + b->off_ctr);
  if (b->persistent) HIP_TRY(b, launch_persist_clear_flag(ctr, b->stream));
  if ((rc = run_seg(b, 0))) return rc;
  for (int i = 0; i + 1 < nsteps; ++i)
    if ((rc = run_seg(b, 1 + (i & 1)))) return rc;
  if ((rc = run_seg(b, 3 + ((nsteps - 1) & 1)))) return rc;
  if ((rc = run_seg(b, 5 + (nsteps & 1)))) return rc;
  if (b->persistent) {  // a dependency wait that ran out leaves the flag set
    uint32_t flag = 0;
    HIP_TRY(b, hipMemcpyAsync(&flag, ctr + 1, sizeof(flag), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    if (flag) return fail(b, ZK_EDEVICE, "persistent batch: a dependency wait ran out");
  }
  return ZK_OK;
}

int zk_batch_autotune(zk_batch *b, double dt, int reps) {
  int rc = check(b);
  if (rc) return rc;
  if (!std::isfinite(dt) || reps < 1) return fail(b, ZK_EINVAL, "bad dt or reps");
  const bool graph = b->use_graph;
  b->use_graph = false;
  b->ready = false;
  b->tune.clear();
  if ((rc = prepare(b, dt))) return rc;
  // keys present in a step, in order of first appearance
  std::vector<Key> keys;
  for (auto &ph : b->seg[1])
    for (auto &l : ph) {
      const Key k{l.row, l.pad, l.nx, l.ny};
      if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
    }
  hipEvent_t e0, e1;
  HIP_TRY(b, hipEventCreate(&e0));
  HIP_TRY(b, hipEventCreate(&e1));
  for (const Key &k : keys) {
    const bool row = std::get<0>(k), pad = std::get<1>(k);
    const int nx = std::get<2>(k), ny = std::get<3>(k);
    float best = 1e30f;
    std::pair<int, int> best_sh = shape_of(b, row, pad, nx, ny);
    for (auto sh : candidates(b, row, pad, row ? nx : ny)) {
      float tot = 0.f;
      for (int r = 0; r <= reps; ++r) {  // r = 0 warms up
        HIP_TRY(b, hipEventRecord(e0, b->stream));
        for (auto &ph : b->seg[1])
          for (BL l : ph) {
            if (l.row != row || l.pad != pad || l.nx != nx || l.ny != ny) continue;
            l.T = sh.first;
            l.E = sh.second;
            l.blocks = blocks_of(row, pad, nx, ny, l.T);
            if ((rc = launch(b, l))) return rc;
          }
        HIP_TRY(b, hipEventRecord(e1, b->stream));
        HIP_TRY(b, hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(b, hipEventElapsedTime(&ms, e0, e1));
        if (r) tot += ms;
      }
      if (tot < best) {
        best = tot;
        best_sh = sh;
      }
    }
    b->tune[k] = best_sh;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  b->use_graph = graph;
  b->ready = false;
  return prepare(b, dt);
}

int zk_batch_tuning(const zk_batch *b, int index, int *row, int *pad, int *n_transform, int *T, int *E) {
  if (!b) return ZK_EINVAL;
  if (index < 0 || index >= (int)b->tune.size()) return ZK_EINVAL;
  auto it = b->tune.begin();
  std::advance(it, index);
  const int r = std::get<0>(it->first), p = std::get<1>(it->first);
  if (row) *row = r;
  if (pad) *pad = p;
  if (n_transform) *n_transform = r ? std::get<2>(it->first) : std::get<3>(it->first);
  if (T) *T = it->second.first;
  if (E) *E = it->second.second;
  return ZK_OK;
}

int zk_batch_stats(const zk_batch *b, long long *phases_per_step, long long *launches_per_step) {
  if (!b) return ZK_EINVAL;
  if (phases_per_step) *phases_per_step = b->phases_per_step;
  if (launches_per_step) *launches_per_step = b->launches_per_step;
  return ZK_OK;
}

const char *zk_batch_last_error(const zk_batch *b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
