// C-ABI of libfind: plan management, footprint/flop queries, and the
// enqueue of a whole FIND solve (procedure computeG<: upward pass, downward
// pass, per-leaf extraction, output collection) on a HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/find.h"
#include "kernels.hpp"
#include "plan.hpp"

using namespace findmi;

namespace {

thread_local std::string g_err;

find_status fail(find_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(FIND_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

struct DevStage {
  int first, count, phase, variant;
  double flops_per_energy;  // algorithmic flops of the stage for one energy
  int rpt;              // panel rows per thread (from the largest front)
  int maxb;             // largest kept set in the stage
  long long ws_stride;  // complex elements per workspace slot
  int maxn;             // largest front in the stage
  ElimDev* d_elims;     // points into DevState::d_elims
};

struct DevState {
  int device = -1;
  int slots = 0;
  size_t mem_total = 0;   // device memory (0: no device to ask)
  ElimDev* d_elims = nullptr;
  int* d_map_node = nullptr;
  int* d_map_srcpos = nullptr;
  LeafOutDev* d_leafout[2] = {nullptr, nullptr};
  int* d_outnode = nullptr;
  int* d_outbond = nullptr;
  std::vector<DevStage> stages;
  int n_leafout[2] = {0, 0};
  double2* pool = nullptr; size_t pool_elems = 0;
  double2* ws = nullptr; size_t ws_elems = 0;
  int* status = nullptr; size_t status_len = 0;
  size_t maps_bytes = 0;
  // profiling: event pairs around stage launches (reused between calls)
  std::vector<hipEvent_t> ev;
  std::vector<double> ev_flops;
  size_t ev_used = 0;
  int launch_count = 0;   // stage launches of the profiled solve
  // concurrent energy groups: one stream and join event per group, one fork event
  std::vector<hipStream_t> lane_st;
  std::vector<hipEvent_t> lane_ev;
  hipEvent_t fork_ev = nullptr;
  // a solve on this device was captured into a graph: buffers the graph
  // references are retired (kept until the plan is destroyed) instead of freed
  bool captured = false;
  std::vector<void*> retired;
};

// Scratch of find_solve_noalloc: a fixed device array (one copy per device,
// held until the process ends) for the energy pool, the elimination
// workspace and the pivot status of that entry point.  Host code never uses
// the array's name as an address: the address of each device's copy comes
// from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kNoAllocScratchBytes = size_t(512) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (set up on first use).
find_status scratch_of(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FIND_E_UNSUPPORTED, "find_solve_noalloc: device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FIND_E_DEVICE, std::string("find_solve_noalloc: hipGetSymbolAddress(scratch): ") +
                                     hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return FIND_OK;
}

__global__ void k_fill_int(int* p, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Node diagonal of the pass's energies into the pool: D[e][0][i] = E_e - H_ii
// - Sigma_d[e][i] (no Sigma_d without scattering) and D[e][1][i] =
// Sigma<_d[e][i] (scattering only); read by the elimination kernels' gathers.
__global__ void k_onsite(StageArgs a) {
  const long long nn = (long long)a.Nx * a.Ny;
  const long long total = nn * a.nE;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int e = int(t / nn);
    const long long i = t - e * nn;
    double2* D = a.pool + (size_t)e * a.pool_stride + a.onsite_off;
    const double2 E = a.energies[e];
    double2 v = make_double2(E.x - a.H[i], E.y);
    if (a.sscat) {
      const double2 sd = a.sscat[e * nn + i];
      v.x -= sd.x; v.y -= sd.y;
      D[nn + i] = a.slscat[e * nn + i];
    }
    D[i] = v;
  }
}

hipError_t launch_onsite(const StageArgs& a, hipStream_t st) {
  const long long total = (long long)a.Nx * a.Ny * a.nE;
  const int grid = int(std::min<long long>((total + 255) / 256, 4096));
  hipLaunchKernelGGL(k_onsite, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace

struct find_plan_s {
  Plan P;
  find_plan_opts opts;
  std::mutex mu;
  std::map<int, std::unique_ptr<DevState>> dev;
  int last_nE = 0;
  int last_device = -1;
  int* last_status = nullptr;  // device pivot-status array of the last solve (last_nE entries)
  bool profiling = false;
  std::vector<int> tiles;      // wave-tile configuration per stage
  std::vector<int> tile_mask;  // bit mask of the configurations each stage has
};

namespace {

void free_dev(DevState& d) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) cur = -1;
  if (d.device >= 0) (void)hipSetDevice(d.device);
  for (hipEvent_t e : d.ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : d.lane_ev) (void)hipEventDestroy(e);
  if (d.fork_ev) (void)hipEventDestroy(d.fork_ev);
  for (hipStream_t s : d.lane_st) (void)hipStreamDestroy(s);
  void* ptrs[] = {d.d_elims, d.d_map_node, d.d_map_srcpos, d.d_leafout[0], d.d_leafout[1],
                  d.d_outnode, d.d_outbond, d.pool, d.ws, d.status};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (void* p : d.retired) (void)hipFree(p);
  if (cur >= 0) (void)hipSetDevice(cur);
}

template <class T>
find_status upload(T** dptr, const std::vector<T>& h, size_t& bytes) {
  size_t nb = std::max<size_t>(1, h.size()) * sizeof(T);
  if (hipMalloc(dptr, nb) != hipSuccess) return fail(FIND_E_NOMEM, "hipMalloc of plan maps failed");
  if (!h.empty()) HIPCHK(hipMemcpy(*dptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  bytes += nb;
  return FIND_OK;
}

// Halved triangles of the symmetric forms, formed and stored as packed lower
// triangles: bit 0 = U (complex symmetric, Prop. 1 of the paper), with
// symmetric = 1 or 2; bit 1 = R (anti-Hermitian), with symmetric = 2 only.
// With symmetric = 1, R is formed and stored whole: the rounding of its two
// computed triangles differs, and replacing one by the mirror of the other
// amplifies the rounding of G< = G R G^dagger by orders of magnitude at
// energies near resonances of the device (where G is large).
int sym_bits(const find_plan_opts& o) { return o.symmetric == 0 ? 0 : o.symmetric == 1 ? 1 : 3; }

// Workspace (complex elements) of one Schur elimination: the tall block
// [A(S,S); A(B,S)] (n x s), L (b x s) and W_q (b x ssig).
long long elim_ws(const Elim& e) {
  return (long long)e.n * e.s + (long long)e.b * e.s + (long long)e.b * e.ssig;
}

// Workgroup slots of a device: workgroups resident per CU (the kernels are
// compiled for occupancy 3; FIND_SLOTS_PER_CU overrides, 1..16) times its
// CUs.  cus < 1 (no device to ask) counts the 256 CUs of an MI355X.
int slots_for(int cus) {
  int per_cu = 3;
  if (const char* env = getenv("FIND_SLOTS_PER_CU")) per_cu = std::max(1, std::min(16, atoi(env)));
  return std::max(1, per_cu * (cus > 0 ? cus : 256));
}

find_status ensure_device(find_plan_s* p, DevState** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  auto it = p->dev.find(dev);
  if (it != p->dev.end()) { *out = it->second.get(); return FIND_OK; }
  auto ds = std::make_unique<DevState>();
  ds->device = dev;
  int cus = 0;
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  ds->slots = slots_for(cus);
  HIPCHK(hipDeviceTotalMem(&ds->mem_total, dev));
  const Plan& P = p->P;
  // elimination records, sorted by decreasing cost inside each stage
  std::vector<ElimDev> he(P.elims.size());
  for (const Stage& st : P.stages) {
    std::vector<int> idx(st.count);
    std::iota(idx.begin(), idx.end(), st.first);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return elim_flops(P.elims[a]) > elim_flops(P.elims[b]); });
    DevStage ds_st{st.first, st.count, st.phase, st.variant, 0.0, 1, 0, 0, 0, nullptr};
    int maxn = 0;
    for (int q = 0; q < st.count; ++q) {
      const Elim& e = P.elims[idx[q]];
      ElimDev& d = he[st.first + q];
      d.kind = e.kind; d.s = e.s; d.b = e.b; d.n = e.n;
      d.src0 = std::max<int64_t>(0, e.src_off[0]); d.src1 = std::max<int64_t>(0, e.src_off[1]);
      d.ld0 = e.src_ld[0]; d.ld1 = e.src_ld[1];
      d.dst = e.dst; d.map = e.map; d.aux = -1; d.rzero = e.rzero; d.ssig = e.ssig; d.bsig = e.bsig; d.bact = e.bact;
      // mixed form: FP32 products except the top-level eliminations, large
      // separators and the final leaf blocks, which stay FP64
      const int top = p->opts.fp64_top_levels == 0 ? 2 : p->opts.fp64_top_levels;
      // bit 0: U product in FP32, bit 1: W and R (Sigma) products in FP32
      const bool low = e.kind == K_SCHUR && e.level > top && e.s < 512;
      d.f32 = !low ? 0 : p->opts.precision == FIND_PREC_MIXED ? 3 : p->opts.precision == FIND_PREC_MIXED_GLESS ? 2 : 0;
      maxn = std::max(maxn, e.n);
      ds_st.maxb = std::max(ds_st.maxb, e.b);
      ds_st.flops_per_energy += elim_flops(e, sym_bits(p->opts));
      const long long need = e.kind == K_FINAL ? 3LL * e.b * e.b  // [U; I] and T
                                               : elim_ws(e);          // tall block, L and W_q
      ds_st.ws_stride = std::max<long long>(ds_st.ws_stride, need);
    }
    if (maxn > kMaxFront) {
      char buf[128];
      snprintf(buf, sizeof buf, "front of size %d exceeds the supported maximum %d", maxn, kMaxFront);
      return fail(FIND_E_UNSUPPORTED, buf);
    }
    ds_st.rpt = panel_rpt(std::max(1, maxn));
    ds_st.maxn = std::max(1, maxn);
    ds->stages.push_back(ds_st);
  }
  std::vector<int> srcpos(P.map_src.size());
  for (size_t k = 0; k < srcpos.size(); ++k)
    srcpos[k] = (P.map_src[k] << 24) | (P.map_src[k] == SRC_ORIG ? 0 : (P.map_pos[k] & 0xffffff));
  std::vector<LeafOutDev> lo[2];
  std::vector<int> elim_to_dev(P.elims.size(), -1);  // plan elimination -> position in he
  for (const Stage& st : P.stages) {
    std::vector<int> idx(st.count);
    std::iota(idx.begin(), idx.end(), st.first);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return elim_flops(P.elims[a]) > elim_flops(P.elims[b]); });
    for (int q = 0; q < st.count; ++q) elim_to_dev[idx[q]] = st.first + q;
  }
  for (const LeafOut& L : P.leafout) {
    he[elim_to_dev[L.elim]].aux = int(lo[L.variant].size());
    const Elim& fe = P.elims[L.elim];
    LeafOutDev d;
    d.elim_dst_lo = int(fe.dst & 0xffffffffLL); d.elim_dst_hi = int(fe.dst >> 32);
    d.bprime = fe.b; d.n_nodes = L.n_nodes; d.node_first = L.node_first;
    d.bond_first = L.bond_first; d.n_bonds = L.n_bonds; d.pad = 0;
    lo[L.variant].push_back(d);
  }
  std::vector<int> onode, obond;
  for (size_t k = 0; k < P.outnode_node.size(); ++k) { onode.push_back(P.outnode_node[k]); onode.push_back(P.outnode_local[k]); }
  for (const OutBond& b : P.outbonds) { obond.push_back(b.bond); obond.push_back(b.li); obond.push_back(b.lj); obond.push_back(b.k); obond.push_back(b.hflat); }
  size_t bytes = 0;
  find_status st;
  if ((st = upload(&ds->d_elims, he, bytes)) != FIND_OK) { free_dev(*ds); return st; }
  if ((st = upload(&ds->d_map_node, P.map_node, bytes)) != FIND_OK) { free_dev(*ds); return st; }
  if ((st = upload(&ds->d_map_srcpos, srcpos, bytes)) != FIND_OK) { free_dev(*ds); return st; }
  for (int v = 0; v < 2; ++v) {
    ds->n_leafout[v] = int(lo[v].size());
    if ((st = upload(&ds->d_leafout[v], lo[v], bytes)) != FIND_OK) { free_dev(*ds); return st; }
  }
  if ((st = upload(&ds->d_outnode, onode, bytes)) != FIND_OK) { free_dev(*ds); return st; }
  if ((st = upload(&ds->d_outbond, obond, bytes)) != FIND_OK) { free_dev(*ds); return st; }
  ds->maps_bytes = bytes;
  for (DevStage& s2 : ds->stages) s2.d_elims = ds->d_elims + s2.first;
  *out = ds.get();
  p->dev[dev] = std::move(ds);
  return FIND_OK;
}

// Workgroups a stage may launch at most: one per slot, or several smaller
// workgroups per slot when its fronts allow the one- or two-wave form.
long long stage_groups(const DevState& d, const DevStage& s) {
  const int g = s.maxn <= kWaveMaxFront ? groups_per_slot(kTileWave)
              : s.maxn <= kTwoWaveMaxFront ? groups_per_slot(kTileTwoWave) : 1;
  return (long long)d.slots * g;
}

// Workspace (complex elements) for passes of ec energies: every stage needs
// one slot per workgroup it launches, min(groups, eliminations x ec).
size_t ws_for(const DevState& d, int ec) {
  size_t w = 0;
  for (const DevStage& s : d.stages)
    w = std::max<size_t>(w, size_t(std::min<long long>(stage_groups(d, s), (long long)s.count * ec)) * s.ws_stride);
  return w;
}

// Energy groups run concurrently (each on its own stream with its own
// workspace) inside one pass.
int lanes_of(const find_plan_s* p) { return std::max(1, std::min(4, p->opts.streams)); }
size_t lane_ws(const DevState& d, int ec, int lanes) { return ws_for(d, (ec + lanes - 1) / lanes); }
size_t ws_total(const DevState& d, int ec, int lanes) { return size_t(lanes) * lane_ws(d, ec, lanes); }

// Device bytes a plan may hold: the caller's budget, else three quarters of
// the device's memory (64 GiB when no device is visible)
size_t budget_of(const find_plan_s* p, const DevState& d) {
  if (p->opts.workspace_budget) return p->opts.workspace_budget;
  return d.mem_total ? d.mem_total / 4 * 3 : (size_t(64) << 30);
}

// energies per internal pass so that pool + workspace fit in the budget
int chunk_energies(const find_plan_s* p, const DevState& d, int nE) {
  const size_t per_e = size_t(p->P.pool_per_energy) * sizeof(double2) + sizeof(int);
  const size_t budget = budget_of(p, d);
  int ec = nE;
  if (p->opts.max_energies > 0) ec = std::min(ec, p->opts.max_energies);
  const int lanes = lanes_of(p);
  auto need = [&](int c) { return ws_total(d, c, lanes) * sizeof(double2) + d.maps_bytes + per_e * size_t(c); };
  while (ec > 1 && need(ec) > budget) ec = std::max(1, std::min(ec - 1, int(ec * double(budget) / double(need(ec)))));
  if (need(ec) > budget) return 0;
  // as many passes as needed, of equal size (a short last pass would leave
  // most of the device idle in the levels with few clusters)
  const int passes = (nE + ec - 1) / ec;
  return (nE + passes - 1) / passes;
}

}  // namespace

// Stage sizes (workspace stride, largest front) and slots of the current
// device (256 CUs if no device is present), as ensure_device sets them,
// without touching device memory.
static void host_stages(const find_plan_s* p, DevState* d) {
  const Plan& P = p->P;
  int dev = -1, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceTotalMem(&d->mem_total, dev) != hipSuccess) {
    (void)hipGetLastError();
    cus = 0;
    d->mem_total = 0;
  }
  d->slots = slots_for(cus);
  for (const Stage& st : P.stages) {
    DevStage ds{st.first, st.count, st.phase, st.variant, 0.0, 1, 0, 0, 1, nullptr};
    for (int k = st.first; k < st.first + st.count; ++k) {
      const Elim& e = P.elims[k];
      ds.ws_stride = std::max<long long>(ds.ws_stride, e.kind == K_FINAL ? 3LL * e.b * e.b : elim_ws(e));
      ds.maxn = std::max(ds.maxn, e.n);
    }
    d->stages.push_back(ds);
  }
}

extern "C" {

const char* find_last_error(void) { return g_err.c_str(); }

int find_n_bonds(int Nx, int Ny, int stencil) {
  if (Nx < 1 || Ny < 1 || (stencil != 5 && stencil != 9)) return -1;
  return count_bonds(Nx, Ny, stencil);
}

find_status find_plan_create(int Nx, int Ny, int stencil, const find_plan_opts* opts, find_plan* out) {
  if (!out) return fail(FIND_E_ARG, "find_plan_create: out is NULL");
  *out = nullptr;
  if (Nx < 1 || Ny < 1) return fail(FIND_E_ARG, "find_plan_create: Nx and Ny must be >= 1");
  if (stencil != 5 && stencil != 9) return fail(FIND_E_ARG, "find_plan_create: stencil must be 5 or 9");
  find_plan_opts o{};
  o.leaf = 8;
  if (opts) o = *opts;
  if (o.leaf == 0) o.leaf = 8;
  if (o.leaf < 1) return fail(FIND_E_ARG, "find_plan_create: leaf must be >= 1");
  if (o.precision != FIND_PREC_FP64 && o.precision != FIND_PREC_MIXED && o.precision != FIND_PREC_MIXED_GLESS)
    return fail(FIND_E_ARG, "find_plan_create: unknown precision");
  if (o.max_energies < 0) return fail(FIND_E_ARG, "find_plan_create: max_energies must be >= 0");
  if (o.complex_mode != FIND_CPLX_4M && o.complex_mode != FIND_CPLX_3M)
    return fail(FIND_E_ARG, "find_plan_create: unknown complex_mode");
  if (o.symmetric < 0 || o.symmetric > 2) return fail(FIND_E_ARG, "find_plan_create: symmetric must be 0, 1 or 2");
  if (o.streams < 0 || o.streams > 4) return fail(FIND_E_ARG, "find_plan_create: streams must be 0..4");
  if (o.scattering != 0 && o.scattering != 1) return fail(FIND_E_ARG, "find_plan_create: scattering must be 0 or 1");
  if (o.half_leaves != 0 && o.half_leaves != 1) return fail(FIND_E_ARG, "find_plan_create: half_leaves must be 0 or 1");
  if (o.no_contacts != 0 && o.no_contacts != 1) return fail(FIND_E_ARG, "find_plan_create: no_contacts must be 0 or 1");
  if ((long long)Nx * Ny > (1LL << 24)) return fail(FIND_E_UNSUPPORTED, "find_plan_create: mesh larger than 2^24 nodes");
  find_plan_s* p = new (std::nothrow) find_plan_s();
  if (!p) return fail(FIND_E_NOMEM, "find_plan_create: host allocation failed");
  p->opts = o;
  std::string err;
  try {
    err = build_plan(Nx, Ny, stencil, o.leaf, p->P, o.scattering != 0, o.half_leaves != 0, o.no_contacts == 0,
                     sym_bits(o));
  } catch (const std::exception& ex) {
    err = std::string("find_plan_create: ") + ex.what();
  }
  if (!err.empty()) { delete p; return fail(FIND_E_ARG, err); }
  if (p->P.max_n > kMaxFront) {
    const int mn = p->P.max_n;
    delete p;
    return fail(FIND_E_UNSUPPORTED, "find_plan_create: largest front has " + std::to_string(mn) +
                                        " nodes, beyond the supported " + std::to_string(kMaxFront));
  }
  for (const Stage& st : p->P.stages) {
    int maxn = 1, maxb = 0, maxrs = 0;
    for (int k = st.first; k < st.first + st.count; ++k) {
      maxn = std::max(maxn, p->P.elims[k].n);
      maxb = std::max(maxb, p->P.elims[k].b);
      maxrs = std::max(maxrs, p->P.elims[k].ssig);
    }
    const bool gj_ok = st.phase == PH_FINAL && st.variant == 0 && maxb <= kGjMaxB && maxrs <= kGjMaxRs;
    const int mask = stage_tile_mask(maxn, st.phase == PH_FINAL, gj_ok);
    if (mask == 0) {
      delete p;
      return fail(FIND_E_UNSUPPORTED, "find_plan_create: a final leaf block of " + std::to_string(maxn / 2) +
                                          " nodes is beyond the supported " + std::to_string(kFourWaveMaxFront / 2));
    }
    // default configuration: the 32x32 wave tile, or the eight-wave form where
    // it is the only one that holds the fronts
    p->tiles.push_back(mask & 1 ? 0 : kTileEight);
    p->tile_mask.push_back(mask);
  }
  *out = p;
  return FIND_OK;
}

find_status find_plan_destroy(find_plan plan) {
  if (!plan) return FIND_OK;
  for (auto& kv : plan->dev) free_dev(*kv.second);
  delete plan;
  return FIND_OK;
}

find_status find_plan_summary(find_plan plan, find_plan_summary_t* out) {
  if (!plan || !out) return fail(FIND_E_ARG, "find_plan_summary: NULL argument");
  const Plan& P = plan->P;
  memset(out, 0, sizeof *out);
  out->Nx = P.Nx; out->Ny = P.Ny; out->stencil = P.stencil; out->leaf = P.leaf;
  out->n_clusters = int(P.cl.size()); out->depth = P.depth; out->n_leaves = P.n_leaves;
  out->n_elims = int(P.elims.size()); out->n_stages = int(P.stages.size());
  out->map_len = int(P.map_node.size());
  out->n_leafout = int(P.leafout.size()); out->n_outbonds = int(P.outbonds.size());
  out->n_outnodes = int(P.outnode_node.size());
  out->max_n = P.max_n; out->max_s = P.max_s; out->max_b = P.max_b;
  out->pool_per_energy = P.pool_per_energy;
  return FIND_OK;
}

find_status find_plan_export(find_plan plan, int32_t* elims, int32_t* maps, int32_t* stages,
                             int32_t* leafout, int32_t* outnodes, int32_t* outbonds) {
  if (!plan) return fail(FIND_E_ARG, "find_plan_export: NULL plan");
  const Plan& P = plan->P;
  if (elims)
    for (size_t k = 0; k < P.elims.size(); ++k) {
      const Elim& e = P.elims[k];
      int32_t* r = elims + k * FIND_EF_FIELDS;
      r[FIND_EF_KIND] = e.kind; r[FIND_EF_S] = e.s; r[FIND_EF_B] = e.b; r[FIND_EF_N] = e.n;
      r[FIND_EF_SRC0] = int32_t(e.src_off[0]); r[FIND_EF_LD0] = e.src_ld[0];
      r[FIND_EF_SRC1] = int32_t(e.src_off[1]); r[FIND_EF_LD1] = e.src_ld[1];
      r[FIND_EF_DST] = int32_t(e.dst); r[FIND_EF_MAP] = e.map;
      r[FIND_EF_CLUSTER] = e.cluster; r[FIND_EF_PHASE] = e.phase; r[FIND_EF_LEVEL] = e.level;
      r[FIND_EF_RZERO] = e.rzero; r[FIND_EF_SSIG] = e.ssig; r[FIND_EF_BSIG] = e.bsig; r[FIND_EF_BACT] = e.bact;
    }
  if (maps)
    for (size_t k = 0; k < P.map_node.size(); ++k) {
      maps[3 * k] = P.map_node[k]; maps[3 * k + 1] = P.map_src[k]; maps[3 * k + 2] = P.map_pos[k];
    }
  if (stages)
    for (size_t k = 0; k < P.stages.size(); ++k) {
      stages[4 * k] = P.stages[k].first; stages[4 * k + 1] = P.stages[k].count;
      stages[4 * k + 2] = P.stages[k].phase; stages[4 * k + 3] = P.stages[k].variant;
    }
  if (leafout)
    for (size_t k = 0; k < P.leafout.size(); ++k) {
      const LeafOut& L = P.leafout[k];
      int32_t* r = leafout + k * FIND_LF_FIELDS;
      r[0] = L.elim; r[1] = L.n_nodes; r[2] = L.node_first; r[3] = L.bond_first; r[4] = L.n_bonds; r[5] = L.variant;
    }
  if (outnodes)
    for (size_t k = 0; k < P.outnode_node.size(); ++k) { outnodes[2 * k] = P.outnode_node[k]; outnodes[2 * k + 1] = P.outnode_local[k]; }
  if (outbonds)
    for (size_t k = 0; k < P.outbonds.size(); ++k) {
      const OutBond& b = P.outbonds[k];
      int32_t* r = outbonds + k * FIND_OB_FIELDS;
      r[0] = b.bond; r[1] = b.li; r[2] = b.lj; r[3] = b.k; r[4] = b.hflat;
    }
  return FIND_OK;
}

find_status find_plan_flops(find_plan plan, int want_bonds, double* flops_per_energy) {
  if (!plan || !flops_per_energy) return fail(FIND_E_ARG, "find_plan_flops: NULL argument");
  const int sb = sym_bits(plan->opts);
  *flops_per_energy = plan->P.flops[sb][want_bonds ? 1 : 0];
  return FIND_OK;
}

find_status find_plan_footprint(find_plan plan, int nE, int want_bonds, size_t* bytes) {
  (void)want_bonds;
  if (!plan || !bytes || nE < 1) return fail(FIND_E_ARG, "find_plan_footprint: bad argument");
  const Plan& P = plan->P;
  // the same sizing find_solve uses, for the current device's slots (if a
  // device is present; else those of an MI355X)
  DevState d;
  host_stages(plan, &d);
  d.maps_bytes = (P.map_node.size() * 2 + P.elims.size() * sizeof(ElimDev) / 4 + P.outbonds.size() * 5 +
                  P.outnode_node.size() * 2) * 4;
  int ec = chunk_energies(plan, d, nE);
  if (ec < 1) ec = 1;
  *bytes = ws_total(d, ec, lanes_of(plan)) * sizeof(double2) + d.maps_bytes +
           (size_t(P.pool_per_energy) * sizeof(double2) + sizeof(int)) * size_t(ec);
  return FIND_OK;
}

}  // extern "C"

namespace {

// Replace a device buffer by a larger one.  Once a solve on this device has
// been captured, the old buffer is retired (kept until the plan is destroyed)
// so that replays of the captured graph still address valid memory.
template <class T>
find_status regrow(DevState* d, T** buf, size_t* have, size_t need, hipStream_t st, const char* what) {
  if (*have >= need) return FIND_OK;
  if (*buf) {
    HIPCHK(hipStreamSynchronize(st));
    if (d->captured) d->retired.push_back(*buf);
    else HIPCHK(hipFree(*buf));
    *buf = nullptr;
    *have = 0;
  }
  if (hipMalloc(buf, need * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    *buf = nullptr;
    return fail(FIND_E_NOMEM, std::string("find_solve: ") + what + " allocation failed");
  }
  *have = need;
  return FIND_OK;
}

// Device buffers for a solve of nE energies (grown on demand); *ec = energies per pass.
// Under stream capture nothing may be allocated: the plan's device state and
// buffers must already be large enough (an eager solve of at least as many
// energies on this device and stream configuration), else FIND_E_ARG.
find_status prepare(find_plan_s* plan, int nE, hipStream_t st, DevState** dout, int* ec) {
  const Plan& P = plan->P;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPCHK(hipStreamIsCapturing(st, &cs));
  const bool capturing = cs != hipStreamCaptureStatusNone;
  DevState* d = nullptr;
  if (capturing) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    auto it = plan->dev.find(dev);
    if (it == plan->dev.end())
      return fail(FIND_E_ARG, "find_solve: captured before an eager solve set the plan up on this device");
    d = it->second.get();
  } else {
    find_status fs = ensure_device(plan, &d);
    if (fs != FIND_OK) return fs;
  }
  *ec = chunk_energies(plan, *d, nE);
  if (*ec < 1) return fail(FIND_E_NOMEM, "find_solve: workspace budget too small for one energy");
  const size_t ws_need = ws_total(*d, *ec, lanes_of(plan));
  const size_t pool_need = size_t(*ec) * size_t(P.pool_per_energy);
  const int lanes = lanes_of(plan);
  if (capturing) {
    if (d->ws_elems < ws_need || d->pool_elems < pool_need || d->status_len < size_t(nE) ||
        (lanes > 1 && (int(d->lane_st.size()) < lanes || !d->fork_ev)))
      return fail(FIND_E_ARG, "find_solve: a captured solve needs buffers that an eager solve of at least as "
                              "many energies has allocated (nothing is allocated under capture)");
    d->captured = true;
    *dout = d;
    return FIND_OK;
  }
  find_status fs;
  if ((fs = regrow(d, &d->ws, &d->ws_elems, ws_need, st, "workspace")) != FIND_OK) return fs;
  if ((fs = regrow(d, &d->pool, &d->pool_elems, pool_need, st, "energy pool")) != FIND_OK) return fs;
  if ((fs = regrow(d, &d->status, &d->status_len, size_t(nE), st, "status")) != FIND_OK) return fs;
  while (int(d->lane_st.size()) < lanes && lanes > 1) {
    hipStream_t s2;
    hipEvent_t e2;
    HIPCHK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));   // default priority
    d->lane_st.push_back(s2);
    HIPCHK(hipEventCreateWithFlags(&e2, hipEventDisableTiming));
    d->lane_ev.push_back(e2);
  }
  if (lanes > 1 && !d->fork_ev) HIPCHK(hipEventCreateWithFlags(&d->fork_ev, hipEventDisableTiming));
  *dout = d;
  return FIND_OK;
}

// Kernel arguments of the pass over energies [e0, e0 + ne).
void pass_args(const find_plan_s* plan, const DevState* d, int variant, int e0, int ne, const double* energies,
               const double* H, const double* sigma, const double* sigma_less, double* diag_G,
               double* diag_Gless, double* bond_G, double* bond_Gless, double* bond_J, StageArgs* pa,
               OutArgs* po, const double* sigma_d = nullptr, const double* sigma_less_d = nullptr,
               const double* sigma_b = nullptr, const double* sigma_less_b = nullptr) {
  const Plan& P = plan->P;
  const size_t nx2 = size_t(P.Nx) * P.Nx;
  const size_t nnodes = size_t(P.Nx) * P.Ny;
  StageArgs a{};
  a.nE = ne;
  a.map_node = d->d_map_node; a.map_srcpos = d->d_map_srcpos;
  a.energies = reinterpret_cast<const double2*>(energies) + e0;
  a.H = H;
  a.sigma = sigma ? reinterpret_cast<const double2*>(sigma) + size_t(e0) * 2 * nx2 : nullptr;
  a.sless = sigma_less ? reinterpret_cast<const double2*>(sigma_less) + size_t(e0) * 2 * nx2 : nullptr;
  a.sscat = sigma_d ? reinterpret_cast<const double2*>(sigma_d) + size_t(e0) * nnodes : nullptr;
  a.slscat = sigma_less_d ? reinterpret_cast<const double2*>(sigma_less_d) + size_t(e0) * nnodes : nullptr;
  // stencil-pattern scattering: [nE][nst-1][Ny][Nx][2] complex per energy
  const size_t bstride = size_t(P.stencil == 9 ? 4 : 2) * nnodes * 2;
  a.sbond = sigma_b ? reinterpret_cast<const double2*>(sigma_b) + size_t(e0) * bstride : nullptr;
  a.slbond = sigma_less_b ? reinterpret_cast<const double2*>(sigma_less_b) + size_t(e0) * bstride : nullptr;
  a.onsite_off = P.onsite_off;
  a.pool = d->pool; a.pool_stride = P.pool_per_energy;
  a.ws = d->ws;   // (an energy group of a multi-stream pass offsets this)
  a.Nx = P.Nx; a.Ny = P.Ny; a.nst = P.stencil == 9 ? 5 : 3;
  a.status = d->status + e0;
  a.sym = sym_bits(plan->opts);
  a.contacts = P.contacts ? 1 : 0;
  OutArgs o{};
  o.leaves = d->d_leafout[variant];
  o.outnode = d->d_outnode; o.outbond = d->d_outbond; o.H = H;
  o.n_bonds = P.n_bonds;
  o.diag_G = reinterpret_cast<double2*>(diag_G) + size_t(e0) * nnodes;
  o.diag_Gless = reinterpret_cast<double2*>(diag_Gless) + size_t(e0) * nnodes;
  o.bond_G = bond_G ? reinterpret_cast<double2*>(bond_G) + size_t(e0) * P.n_bonds : nullptr;
  o.bond_Gless = bond_Gless ? reinterpret_cast<double2*>(bond_Gless) + size_t(e0) * P.n_bonds : nullptr;
  o.bond_J = bond_J ? bond_J + size_t(e0) * P.n_bonds : nullptr;
  *pa = a;
  *po = o;
}

// Launch stage k of a pass with wave-tile configuration tc; grid < 1 = nothing to do.
hipError_t launch_stage_k(const find_plan_s* plan, const DevState* d, int k, StageArgs a, const OutArgs& o,
                          int tc, hipStream_t st) {
  const DevStage& s2 = d->stages[k];
  a.elims = s2.d_elims; a.n_elims = s2.count; a.ws_stride = s2.ws_stride;
  const long long items = (long long)s2.count * a.nE;
  const long long groups = stage_grid_groups(d->slots, tc);
  const int grid = int(std::min<long long>(items, groups));
  if (grid < 1) return hipSuccess;
  if (s2.phase == PH_FINAL) return launch_final_tc(a, o, s2.maxn, tc, grid, st);
  return launch_stage(a, s2.maxn, tc, plan->opts.complex_mode, grid, st);
}

// Device buffers a solve runs in: the energy pool (ec energies), the
// elimination workspace (lanes groups of lane_ws elements) and the per-energy
// pivot status (nE entries).
struct SolveBufs {
  double2* pool;
  double2* ws;
  int* status;
  int ec;
  int lanes;
  size_t lane_ws;
  bool profiling;
};

// Enqueue every pass of a solve into `b` on `st`; arguments checked by the callers.
find_status enqueue_solve(find_plan plan, DevState* d, const SolveBufs& b, int nE, const double* energies,
                          const double* H, const double* sigma, const double* sigma_less, const double* sigma_d,
                          const double* sigma_less_d, double* diag_G, double* diag_Gless, double* bond_G,
                          double* bond_Gless, double* bond_J, hipStream_t st, const double* sigma_b = nullptr,
                          const double* sigma_less_b = nullptr) {
  const int variant = (bond_G || bond_Gless || bond_J) ? 1 : 0;
  if (b.profiling) { d->ev_used = 0; d->launch_count = 0; }  // the profile describes this solve
  hipLaunchKernelGGL(k_fill_int, dim3((nE + 255) / 256), dim3(256), 0, st, b.status, nE, 0);
  HIPCHK(hipGetLastError());
  const int ec = b.ec, lanes = b.lanes;
  const size_t lws = b.lane_ws;
  for (int e0 = 0; e0 < nE; e0 += ec) {
    const int ne = std::min(ec, nE - e0);
    // energy groups of this pass: one on the caller's stream, or `lanes`
    // groups on the plan's streams, forked from and joined back to it
    const int ng = (lanes > 1 && ne > 1) ? std::min(lanes, ne) : 1;
    const int per = (ne + ng - 1) / ng;
    if (ng > 1) {
      if (b.profiling) {   // one event pair around the whole pass
        while (d->ev.size() < 2 * (d->ev_used + 1)) {
          hipEvent_t ev;
          HIPCHK(hipEventCreate(&ev));
          d->ev.push_back(ev);
        }
        if (d->ev_flops.size() < d->ev_used + 1) d->ev_flops.resize(d->ev_used + 1);
        double f = 0.0;
        for (const DevStage& s2 : d->stages)
          if (s2.variant < 0 || s2.variant == variant) f += s2.flops_per_energy * ne;
        d->ev_flops[d->ev_used] = f;
        HIPCHK(hipEventRecord(d->ev[2 * d->ev_used], st));
      }
      HIPCHK(hipEventRecord(d->fork_ev, st));
    }
    for (int g = 0; g < ng; ++g) {
      const int g0 = e0 + g * per, gn = std::min(per, e0 + ne - g0);
      if (gn < 1) continue;
      hipStream_t sg = ng > 1 ? d->lane_st[g] : st;
      if (ng > 1) HIPCHK(hipStreamWaitEvent(sg, d->fork_ev, 0));
      StageArgs a;
      OutArgs o;
      pass_args(plan, d, variant, g0, gn, energies, H, sigma, sigma_less, diag_G, diag_Gless, bond_G, bond_Gless,
                bond_J, &a, &o, sigma_d, sigma_less_d, sigma_b, sigma_less_b);
      a.ws = b.ws + size_t(g) * lws;
      a.pool = b.pool + size_t(g0 - e0) * size_t(plan->P.pool_per_energy);   // kernels index energies from 0
      a.status = b.status + g0;
      {
        const hipError_t he = launch_onsite(a, sg);
        if (he != hipSuccess) return fail(FIND_E_DEVICE, std::string("onsite launch: ") + hipGetErrorString(he));
      }
      for (size_t k = 0; k < d->stages.size(); ++k) {
        const DevStage& s2 = d->stages[k];
        if (s2.variant >= 0 && s2.variant != variant) continue;
        if ((long long)s2.count * gn < 1) continue;
        const bool prof = b.profiling && ng == 1;
        if (prof) {
          while (d->ev.size() < 2 * (d->ev_used + 1)) {
            hipEvent_t ev;
            HIPCHK(hipEventCreate(&ev));
            d->ev.push_back(ev);
          }
          if (d->ev_flops.size() < d->ev_used + 1) d->ev_flops.resize(d->ev_used + 1);
          d->ev_flops[d->ev_used] = s2.flops_per_energy * gn;
          HIPCHK(hipEventRecord(d->ev[2 * d->ev_used], sg));
        }
        // solves with stencil-pattern scattering self-energies run the
        // configurations compiled with the bond reads (the 32x32 wave tile of
        // the one-, two-, four- and eight-wave forms): the stage's own where
        // it is one of them, else configuration 0 (the eight-wave form where
        // it is the only one)
        const int tk = plan->tiles[k];
        const bool bond_cfg = tk == 0 || tk == kTileWave || tk == kTileTwoWave || tk == kTileEight;
        const int tck = (a.sbond && s2.phase != PH_FINAL && !bond_cfg)
                            ? ((plan->tile_mask[k] & 1) ? 0 : kTileEight) : tk;
        const hipError_t he = launch_stage_k(plan, d, int(k), a, o, tck, sg);
        if (he != hipSuccess) return fail(FIND_E_DEVICE, std::string("stage launch: ") + hipGetErrorString(he));
        if (b.profiling) ++d->launch_count;
        if (prof) {
          HIPCHK(hipEventRecord(d->ev[2 * d->ev_used + 1], sg));
          ++d->ev_used;
        }
      }
      if (ng > 1) {
        HIPCHK(hipEventRecord(d->lane_ev[g], sg));
        HIPCHK(hipStreamWaitEvent(st, d->lane_ev[g], 0));
      }
    }
    if (ng > 1 && b.profiling) {
      HIPCHK(hipEventRecord(d->ev[2 * d->ev_used + 1], st));
      ++d->ev_used;
    }
  }
  plan->last_nE = nE;
  plan->last_device = d->device;
  plan->last_status = b.status;
  return FIND_OK;
}

// The solve of find_solve and find_solve_scattering(_bonds) (the scattering
// arrays NULL where absent) in the plan's own buffers; arguments checked by
// the callers.
find_status solve_impl(find_plan plan, int nE, const double* energies, const double* H, const double* sigma,
                       const double* sigma_less, const double* sigma_d, const double* sigma_less_d,
                       double* diag_G, double* diag_Gless,
                       double* bond_G, double* bond_Gless, double* bond_J, void* hip_stream,
                       const double* sigma_b = nullptr, const double* sigma_less_b = nullptr) {
  std::lock_guard<std::mutex> lk(plan->mu);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  plan->last_status = nullptr;
  plan->last_nE = 0;
  DevState* d = nullptr;
  int ec = 0;
  find_status fs = prepare(plan, nE, st, &d, &ec);
  if (fs != FIND_OK) return fs;
  const int lanes = lanes_of(plan);
  const SolveBufs b{d->pool, d->ws, d->status, ec, lanes, lane_ws(*d, ec, lanes), plan->profiling};
  return enqueue_solve(plan, d, b, nE, energies, H, sigma, sigma_less, sigma_d, sigma_less_d, diag_G, diag_Gless,
                       bond_G, bond_Gless, bond_J, st, sigma_b, sigma_less_b);
}

}  // namespace

extern "C" {

find_status find_solve(find_plan plan, int nE, const double* energies, const double* H, const double* sigma,
                       const double* sigma_less, double* diag_G, double* diag_Gless, double* bond_G,
                       double* bond_Gless, double* bond_J, void* hip_stream) {
  if (!plan) return fail(FIND_E_ARG, "find_solve: NULL plan");
  if (nE < 1) return fail(FIND_E_ARG, "find_solve: nE must be >= 1");
  if (!energies || !H || !diag_G || !diag_Gless || (plan->P.contacts && (!sigma || !sigma_less)))
    return fail(FIND_E_ARG, "find_solve: NULL input or diagonal output pointer");
  if (plan->opts.scattering)
    return fail(FIND_E_ARG, "find_solve: the plan expects scattering self-energies (find_solve_scattering)");
  return solve_impl(plan, nE, energies, H, sigma, sigma_less, nullptr, nullptr, diag_G, diag_Gless, bond_G,
                    bond_Gless, bond_J, hip_stream);
}

find_status find_solve_scattering(find_plan plan, int nE, const double* energies, const double* H,
                                  const double* sigma, const double* sigma_less, const double* sigma_d,
                                  const double* sigma_less_d, double* diag_G, double* diag_Gless,
                                  double* bond_G, double* bond_Gless, double* bond_J, void* hip_stream) {
  if (!plan) return fail(FIND_E_ARG, "find_solve_scattering: NULL plan");
  if (nE < 1) return fail(FIND_E_ARG, "find_solve_scattering: nE must be >= 1");
  if (!energies || !H || !sigma_d || !sigma_less_d || !diag_G || !diag_Gless ||
      (plan->P.contacts && (!sigma || !sigma_less)))
    return fail(FIND_E_ARG, "find_solve_scattering: NULL input or diagonal output pointer");
  if (!plan->opts.scattering)
    return fail(FIND_E_ARG, "find_solve_scattering: the plan was created without opts.scattering");
  return solve_impl(plan, nE, energies, H, sigma, sigma_less, sigma_d, sigma_less_d, diag_G, diag_Gless, bond_G,
                    bond_Gless, bond_J, hip_stream);
}

find_status find_solve_scattering_bonds(find_plan plan, int nE, const double* energies, const double* H,
                                        const double* sigma, const double* sigma_less, const double* sigma_d,
                                        const double* sigma_less_d, const double* sigma_b,
                                        const double* sigma_less_b, double* diag_G, double* diag_Gless,
                                        double* bond_G, double* bond_Gless, double* bond_J, void* hip_stream) {
  if (!plan) return fail(FIND_E_ARG, "find_solve_scattering_bonds: NULL plan");
  if (nE < 1) return fail(FIND_E_ARG, "find_solve_scattering_bonds: nE must be >= 1");
  if (!energies || !H || !sigma_d || !sigma_less_d || !sigma_b || !sigma_less_b || !diag_G || !diag_Gless ||
      (plan->P.contacts && (!sigma || !sigma_less)))
    return fail(FIND_E_ARG, "find_solve_scattering_bonds: NULL input or diagonal output pointer");
  if (!plan->opts.scattering)
    return fail(FIND_E_ARG, "find_solve_scattering_bonds: the plan was created without opts.scattering");
  if (plan->opts.complex_mode != FIND_CPLX_4M)
    return fail(FIND_E_UNSUPPORTED, "find_solve_scattering_bonds: 4M complex products only");
  return solve_impl(plan, nE, energies, H, sigma, sigma_less, sigma_d, sigma_less_d, diag_G, diag_Gless, bond_G,
                    bond_Gless, bond_J, hip_stream, sigma_b, sigma_less_b);
}

find_status find_solve_noalloc(find_plan plan, int nE, const double* energies, const double* H,
                               const double* sigma, const double* sigma_less, double* diag_G, double* diag_Gless,
                               double* bond_G, double* bond_Gless, double* bond_J, void* hip_stream) {
  if (!plan) return fail(FIND_E_ARG, "find_solve_noalloc: NULL plan");
  if (nE < 1) return fail(FIND_E_ARG, "find_solve_noalloc: nE must be >= 1");
  if (!energies || !H || !diag_G || !diag_Gless || (plan->P.contacts && (!sigma || !sigma_less)))
    return fail(FIND_E_ARG, "find_solve_noalloc: NULL input or diagonal output pointer");
  if (plan->opts.scattering)
    return fail(FIND_E_ARG, "find_solve_noalloc: scattering plans are not supported (use find_solve_scattering)");
  std::lock_guard<std::mutex> lk(plan->mu);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  plan->last_status = nullptr;
  plan->last_nE = 0;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  auto it = plan->dev.find(dev);
  DevState* d = it == plan->dev.end() ? nullptr : it->second.get();
  DevState sizing;                       // (host copy of the stage sizes if the plan is not on the device)
  if (!d) host_stages(plan, &sizing);
  const DevState& z = d ? *d : sizing;
  // largest pass that fits: status (nE ints), pool (ec energies), workspace (ec energies, one group)
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t per_e = size_t(plan->P.pool_per_energy) * sizeof(double2);
  const size_t st_bytes = up(size_t(nE) * sizeof(int));
  auto need = [&](int c) { return st_bytes + up(per_e * size_t(c)) + ws_for(z, c) * sizeof(double2); };
  int ec = nE;
  if (plan->opts.max_energies > 0) ec = std::min(ec, plan->opts.max_energies);
  while (ec > 1 && need(ec) > kNoAllocScratchBytes)
    ec = std::max(1, std::min(ec - 1, int(ec * double(kNoAllocScratchBytes) / double(need(ec)))));
  if (need(ec) > kNoAllocScratchBytes) {
    char buf[200];
    snprintf(buf, sizeof buf, "find_solve_noalloc: one energy of this plan needs %zu bytes of scratch, "
             "more than the %zu the library holds per device", need(1), kNoAllocScratchBytes);
    return fail(FIND_E_NOMEM, buf);
  }
  if (!d)
    return fail(FIND_E_ARG, "find_solve_noalloc: the plan has no tables on this device "
                            "(run find_solve with it once on this device first)");
  unsigned char* base = nullptr;
  find_status fs = scratch_of(dev, &base);
  if (fs != FIND_OK) return fs;
  int* status = reinterpret_cast<int*>(base);
  double2* pool = reinterpret_cast<double2*>(base + st_bytes);
  double2* ws = reinterpret_cast<double2*>(base + st_bytes + up(per_e * size_t(ec)));
  const SolveBufs b{pool, ws, status, ec, 1, ws_for(*d, ec), false};
  return enqueue_solve(plan, d, b, nE, energies, H, sigma, sigma_less, nullptr, nullptr, diag_G, diag_Gless,
                       bond_G, bond_Gless, bond_J, st);
}

find_status find_plan_autotune(find_plan plan, int nE, const double* energies, const double* H,
                               const double* sigma, const double* sigma_less, double* diag_G,
                               double* diag_Gless, int reps, void* hip_stream) {
  if (!plan) return fail(FIND_E_ARG, "find_plan_autotune: NULL plan");
  if (nE < 1) return fail(FIND_E_ARG, "find_plan_autotune: nE must be >= 1");
  if (!energies || !H || !diag_G || !diag_Gless || (plan->P.contacts && (!sigma || !sigma_less)))
    return fail(FIND_E_ARG, "find_plan_autotune: NULL input or output pointer");
  if (reps < 1) reps = 2;
  std::lock_guard<std::mutex> lk(plan->mu);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPCHK(hipStreamIsCapturing(st, &cs));
  if (cs != hipStreamCaptureStatusNone) return fail(FIND_E_ARG, "find_plan_autotune: stream is being captured");
  DevState* d = nullptr;
  int ec = 0;
  find_status fs = prepare(plan, nE, st, &d, &ec);
  if (fs != FIND_OK) return fs;
  const int ne = std::min(ec, nE);
  hipLaunchKernelGGL(k_fill_int, dim3((ne + 255) / 256), dim3(256), 0, st, d->status, ne, 0);
  HIPCHK(hipGetLastError());
  StageArgs a;
  OutArgs o;
  pass_args(plan, d, 0, 0, ne, energies, H, sigma, sigma_less, diag_G, diag_Gless, nullptr, nullptr, nullptr, &a, &o);
  if (launch_onsite(a, st) != hipSuccess) return fail(FIND_E_DEVICE, "find_plan_autotune: onsite launch");
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  find_status res = FIND_OK;
  for (size_t k = 0; k < d->stages.size() && res == FIND_OK; ++k) {
    const DevStage& s2 = d->stages[k];
    if (s2.variant >= 0 && s2.variant != 0) continue;
    const int mask = plan->tile_mask[k];
    const bool several = (mask & (mask - 1)) != 0;
    int best = plan->tiles[k], last = -1;
    float best_ms = -1.f;
    for (int tc = 0; tc < kTileConfigs && res == FIND_OK; ++tc) {
      if (!(mask >> tc & 1)) continue;
      // a first untimed launch (it also leaves the stage's outputs for the next stage)
      hipError_t he = launch_stage_k(plan, d, int(k), a, o, tc, st);
      if (he == hipSuccess && several) {
        he = hipEventRecord(e0, st);
        for (int r = 0; r < reps && he == hipSuccess; ++r) he = launch_stage_k(plan, d, int(k), a, o, tc, st);
        if (he == hipSuccess) he = hipEventRecord(e1, st);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he == hipSuccess && (best_ms < 0.f || ms < best_ms)) { best_ms = ms; best = tc; }
      }
      if (he != hipSuccess) res = fail(FIND_E_DEVICE, std::string("find_plan_autotune: ") + hipGetErrorString(he));
      last = tc;
    }
    // leave the chosen configuration's outputs for the next stage (configurations
    // may round differently), so that the pass equals a solve with the chosen tiles
    if (res == FIND_OK && last != best) {
      const hipError_t he = launch_stage_k(plan, d, int(k), a, o, best, st);
      if (he != hipSuccess) res = fail(FIND_E_DEVICE, std::string("find_plan_autotune: ") + hipGetErrorString(he));
    }
    plan->tiles[k] = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (res != FIND_OK) return res;
  HIPCHK(hipStreamSynchronize(st));
  plan->last_nE = ne;
  plan->last_device = d->device;
  plan->last_status = d->status;
  return FIND_OK;
}

find_status find_plan_get_tiles(find_plan plan, int* tiles, int* masks, int cap, int* n_stages) {
  if (!plan) return fail(FIND_E_ARG, "find_plan_get_tiles: NULL plan");
  std::lock_guard<std::mutex> lk(plan->mu);
  const int n = int(plan->tiles.size());
  if (n_stages) *n_stages = n;
  for (int k = 0; k < std::min(n, cap); ++k) {
    if (tiles) tiles[k] = plan->tiles[k];
    if (masks) masks[k] = plan->tile_mask[k];
  }
  return FIND_OK;
}

find_status find_plan_set_tiles(find_plan plan, const int* tiles, int n) {
  if (!plan || !tiles) return fail(FIND_E_ARG, "find_plan_set_tiles: NULL argument");
  std::lock_guard<std::mutex> lk(plan->mu);
  if (n != int(plan->tiles.size())) return fail(FIND_E_ARG, "find_plan_set_tiles: n must equal the stage count");
  for (int k = 0; k < n; ++k)
    if (tiles[k] < 0 || tiles[k] >= kTileConfigs || !(plan->tile_mask[k] >> tiles[k] & 1))
      return fail(FIND_E_ARG, "find_plan_set_tiles: stage " + std::to_string(k) + " has no configuration " +
                                  std::to_string(tiles[k]));
  for (int k = 0; k < n; ++k) plan->tiles[k] = tiles[k];
  return FIND_OK;
}

find_status find_plan_set_profiling(find_plan plan, int enable) {
  if (!plan) return fail(FIND_E_ARG, "find_plan_set_profiling: NULL plan");
  std::lock_guard<std::mutex> lk(plan->mu);
  plan->profiling = enable != 0;
  return FIND_OK;
}

find_status find_plan_profile(find_plan plan, double* kernel_ms, double* kernel_flops, int* launches) {
  if (!plan) return fail(FIND_E_ARG, "find_plan_profile: NULL plan");
  std::lock_guard<std::mutex> lk(plan->mu);
  double ms = 0.0, fl = 0.0;
  int nl = 0;
  for (auto& kv : plan->dev) {
    DevState& d = *kv.second;
    for (size_t k = 0; k < d.ev_used; ++k) {
      HIPCHK(hipEventSynchronize(d.ev[2 * k + 1]));
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, d.ev[2 * k], d.ev[2 * k + 1]));
      ms += t;
      fl += d.ev_flops[k];
    }
    nl += d.launch_count;
  }
  if (kernel_ms) *kernel_ms = ms;
  if (kernel_flops) *kernel_flops = fl;
  if (launches) *launches = nl;
  return FIND_OK;
}

find_status find_sync_status(find_plan plan, void* hip_stream) {
  if (!plan) return fail(FIND_E_ARG, "find_sync_status: NULL plan");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  HIPCHK(hipStreamSynchronize(st));
  std::lock_guard<std::mutex> lk(plan->mu);
  if (!plan->last_status || plan->last_nE == 0) return FIND_OK;
  std::vector<int> h(plan->last_nE);
  HIPCHK(hipMemcpy(h.data(), plan->last_status, h.size() * sizeof(int), hipMemcpyDeviceToHost));
  for (size_t e = 0; e < h.size(); ++e)
    if (h[e]) {
      char buf[96];
      snprintf(buf, sizeof buf, "zero or tiny pivot (|pivot| < 1e3 eps max|A(S,S)|) met at energy index %zu", e);
      return fail(FIND_E_SINGULAR, buf);
    }
  return FIND_OK;
}

}  // extern "C"
