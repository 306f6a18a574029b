// Host side of libwc: contexts, batches of lattices, the FGCR driver and the C interface.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "wc.h"
#include "dense_host.h"
#include "wc_kernels.h"

namespace wc {

void launch_force(const int* L, int bc_t, const void* Ucanon, const void* Y, const void* X, int nrhs, double csw,
                  double coef, int out_kind, void* xi_work, void* out, hipStream_t st);
void launch_gamma5_canon(long long nsite, const void* src, void* dst, hipStream_t st);
void launch_gamma5_f64(void* f, long long V, int nrhs, hipStream_t st);
void launch_clover_export(const Geom& g, const void* c64, void* out, hipStream_t st);
void launch_fill_hash(long long n, unsigned seed, void* out, hipStream_t st);
void launch_scale_canon(long long n, double coef, const void* in, void* out, hipStream_t st);
void launch_norm2_canon(long long n, const void* v, double* work, hipStream_t st);
static_assert(HIST_MAX == WC_HIST_MAX, "history length of the device state and the interface");

struct Error {
  int code;
  std::string msg;
};

thread_local std::string g_last_error;

#define HIPCK(expr)                                                                                    \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess)                                                                              \
      throw Error{e_ == hipErrorOutOfMemory ? WC_ERR_OOM : WC_ERR_HIP,                                 \
                  std::string(#expr) + ": " + hipGetErrorString(e_)};                                  \
  } while (0)

static void require(bool ok, int code, const std::string& msg) {
  if (!ok) throw Error{code, msg};
}

// HIP event released on every exit path (HIPCK throws)
struct HipEvent {
  hipEvent_t e = nullptr;
  HipEvent() { HIPCK(hipEventCreate(&e)); }
  ~HipEvent() {
    if (e) (void)hipEventDestroy(e);
  }
  HipEvent(const HipEvent&) = delete;
  HipEvent& operator=(const HipEvent&) = delete;
  operator hipEvent_t() const { return e; }
};

// Instantiated graph of what f enqueues on the capture stream `cap`.  If f throws, the
// capture is ended and its partial graph dropped, so `cap` leaves capture mode.
static hipGraphExec_t capture_graph(hipStream_t cap, const std::function<void(hipStream_t)>& f) {
  HIPCK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  try {
    f(cap);
  } catch (...) {
    hipGraph_t partial = nullptr;
    if (hipStreamEndCapture(cap, &partial) == hipSuccess && partial) (void)hipGraphDestroy(partial);
    throw;
  }
  hipGraph_t graph;
  HIPCK(hipStreamEndCapture(cap, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t instantiate = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCK(instantiate);
  return exec;
}

// owning device allocation
struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void ensure(size_t bytes) {
    if (bytes <= n && p) return;
    release();
    HIPCK(hipMalloc(&p, bytes ? bytes : 16));
    n = bytes;
  }
  template <class T> T* as() const { return (T*)p; }
};

static int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

static int persistent_grid(int nitems, int per_cu) {
  const int cap = device_cus() * per_cu;
  return std::max(1, std::min(nitems, cap));
}

static bool valid_block(const int* L, const int* b) {
  int vol = 1;
  for (int m = 0; m < 4; ++m) {
    if (b[m] <= 0 || L[m] % b[m] || (L[m] / b[m]) % 2) return false;
    vol *= b[m];
  }
  return vol <= 256;
}

static Geom make_geom(const int* L, const int* B, int bc_t) {
  Geom g;
  for (int m = 0; m < 4; ++m) {
    g.L[m] = L[m];
    g.B[m] = B[m];
    g.NB[m] = L[m] / B[m];
  }
  g.lstr[3] = 1;
  g.lstr[2] = B[3];
  g.lstr[1] = B[3] * B[2];
  g.lstr[0] = B[3] * B[2] * B[1];
  g.tstr[3] = 1;
  g.tstr[2] = g.NB[3];
  g.tstr[1] = g.NB[3] * g.NB[2];
  g.tstr[0] = g.NB[3] * g.NB[2] * g.NB[1];
  g.bvol = B[0] * B[1] * B[2] * B[3];
  g.ntiles = g.NB[0] * g.NB[1] * g.NB[2] * g.NB[3];
  g.V = L[0] * L[1] * L[2] * L[3];
  g.bc_t = bc_t;
  return g;
}

static size_t spinor_bytes(int prec, long long sites_rhs) { return (size_t)sites_rhs * spinor_site_bytes(prec); }
static bool is16(int prec) { return prec == P_F16 || prec == P_BF16; }

// A spinor field in a storage precision: data + optional 16-bit scales.
struct Field {
  DevBuf d, sc;
  int prec = -1;
  long long n = 0;
  void ensure(int p, long long sites_rhs) {
    if (prec == p && n >= sites_rhs && d.p) return;
    d.ensure(spinor_bytes(p, sites_rhs));
    if (is16(p)) sc.ensure(sizeof(float) * sites_rhs);
    prec = p;
    n = sites_rhs;
  }
  void* data() const { return d.p; }
  float* scale() const { return is16(prec) ? sc.as<float>() : nullptr; }
};

struct Batch;

// ---------------------------------------------------------------------------- allocation-free scratch

// Device memory of wc_apply_D_noalloc: a fixed array in the library's code object, one copy
// per GPU, held until the process ends.  Host code never names it in device work: it uses
// the per-device address that scratch_setup() obtains from the runtime.
constexpr size_t SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int SCRATCH_MAX_DEVICES = 64;
static void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

// Address of this device's scratch array (the device must be current); resolved once per
// device, at the first context created on it.
static void* scratch_setup(int dev) {
  require(dev >= 0 && dev < SCRATCH_MAX_DEVICES, WC_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    require(ptr != nullptr, WC_ERR_HIP, "scratch array has no device address");
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace wc

struct wc_ctx {
  int dev = 0;
  wc::Geom g;
  int dims[4];
  int block[4];
  int bc_t = 1;
  double m0 = 0, csw = 0;
  bool have_clover = false;
  wc::DevBuf Ucanon;
  wc::DevBuf links[4], lscale[4];
  bool have_links[4] = {false, false, false, false};
  wc::DevBuf clov[4], cscale[4];
  bool have_clov[4] = {false, false, false, false};
  wc::DevBuf clov_eo[4], cscale_eo[4];  // even/odd block solver: A on even, A^-1 on odd sites
  bool have_clov_eo[4] = {false, false, false, false};
  wc::DevBuf tiles[2];
  wc::DevBuf eo_sites;                    // [corner parity][site parity][(bvol+1)/2] local indices
  wc::DevBuf eo_slot;                     // [corner parity][bvol] parity-sorted slot of each local site
  int nr_dirac[4] = {0, 0, 0, 0};
  int nr_sap[4] = {0, 0, 0, 0};
  int nr_sap_eo[4] = {0, 0, 0, 0};
  int opt_sap_cache = -1;    // WC_OPT_SAP_CACHE: -1 automatic, 0 reload, 1 registers
  int opt_dirac_stage = -1;  // WC_OPT_DIRAC_STAGE: -1 automatic, 0 off, 1 on
  std::map<int, std::unique_ptr<wc::Batch>> batches;  // single-lattice batches by nrhs
  hipStream_t cap = nullptr;                           // capture stream for graphs
  ~wc_ctx();
};

namespace wc {

static void ensure_links(wc_ctx* c, int prec, hipStream_t st) {
  if (c->have_links[prec]) return;
  c->links[prec].ensure((size_t)c->g.V * link_site_bytes(prec) + (is16(prec) ? 0 : 0));
  if (is16(prec)) c->lscale[prec].ensure(sizeof(float) * c->g.V);
  launch_pack_links(prec, c->g, c->Ucanon.p, c->links[prec].p, c->lscale[prec].as<float>(), st);
  HIPCK(hipGetLastError());
  c->have_links[prec] = true;
}

static void ensure_clover(wc_ctx* c, int prec, hipStream_t st) {
  require(c->have_clover, WC_ERR_STATE, "clover term not created (call wc_create_clover)");
  if (c->have_clov[prec]) return;
  c->clov[prec].ensure((size_t)c->g.V * clover_site_bytes(prec));
  if (is16(prec)) c->cscale[prec].ensure(sizeof(float) * 2 * c->g.V);
  launch_clover_convert(prec, c->g, c->clov[P_F64].p, c->clov[prec].p, c->cscale[prec].as<float>(), st);
  HIPCK(hipGetLastError());
  c->have_clov[prec] = true;
}

static void ensure_clover_eo(wc_ctx* c, int prec, hipStream_t st) {
  require(c->have_clover, WC_ERR_STATE, "clover term not created (call wc_create_clover)");
  if (c->have_clov_eo[prec]) return;
  if (!c->have_clov_eo[P_F64]) {
    c->clov_eo[P_F64].ensure((size_t)c->g.V * clover_site_bytes(P_F64));
    launch_clover_eo(c->g, c->clov[P_F64].p, c->clov_eo[P_F64].p, st);
    HIPCK(hipGetLastError());
    c->have_clov_eo[P_F64] = true;
  }
  if (prec != P_F64) {
    c->clov_eo[prec].ensure((size_t)c->g.V * clover_site_bytes(prec));
    if (is16(prec)) c->cscale_eo[prec].ensure(sizeof(float) * 2 * c->g.V);
    launch_clover_convert(prec, c->g, c->clov_eo[P_F64].p, c->clov_eo[prec].p, c->cscale_eo[prec].as<float>(), st);
    HIPCK(hipGetLastError());
    c->have_clov_eo[prec] = true;
  }
}

// ---------------------------------------------------------------------------- batches

struct ItemList {
  DevBuf d;
  int n = 0;
};

struct Batch {
  std::vector<wc_ctx*> lat;
  std::vector<int> nrhs;
  int nsys = 0;
  long long sites_rhs = 0;
  int total_chunks = 0;
  int max_bvol = 0;
  int uniform_bvol = 0;  // block volume shared by all lattices, 0 if they differ
  std::vector<LatDesc> h_lats[4];
  DevBuf d_lats[4];
  bool have_lats[4] = {false, false, false, false};
  bool lats_eo[4] = {false, false, false, false};  // descriptors carry the even/odd clover
  std::map<int, ItemList> dirac_items;      // by RHS tile
  std::map<int, ItemList> sap_items[2];     // by RHS tile and block volume
  DevBuf sys_part, sys_nchunks;
  DevBuf partials;
  int pw = 4 * NKV_MAX;  // partial-sum width (at most RWG: sum_partials)
  // solver state
  Field x, b, r, chi[NKV_MAX], phi[NKV_MAX];
  Field w;    // FGCR with an F32 basis: the direction D phi_k (F32) before its Gram-Schmidt
  Field r32;  // ... and the recursion's residual between restarts (F32)
  DevBuf dead;  // FGCR: cycle-ended flag and the counts behind it (VecLaunch::dead)
  DevBuf d_chi, d_phi;
  // FGCR directions in the preconditioner's storage, and their pointer tables
  Field dir[NKV_MAX];
  DevBuf d_dir, d_dir_sc;
  Field sap_rho, sap_z, sap_psi;
  DevBuf sys, skip;
  DevBuf hist;  // [nsys][HIST_MAX] relative true residual after each restart
  // apply / bench buffers per precision
  Field ain[4], aout[4];
  // captured restart cycle
  hipGraphExec_t graph = nullptr;
  std::string graph_key;
  // FGMRES-DR: the last basis vector V_m, the basis pointer table (m+1 entries), the
  // per-system cycle state and the captured cycles by (setup, first column)
  Field arn_vlast;
  DevBuf d_arn_v, arn;
  std::map<std::string, hipGraphExec_t> arn_graphs;
  std::string arn_key;  // graph_key the graphs in arn_graphs were captured under

  ~Batch() {
    if (graph) (void)hipGraphExecDestroy(graph);
    for (auto& kv : arn_graphs) (void)hipGraphExecDestroy(kv.second);
  }

  void init(const std::vector<wc_ctx*>& l, const std::vector<int>& n) {
    lat = l;
    nrhs = n;
    nsys = 0;
    sites_rhs = 0;
    total_chunks = 0;
    max_bvol = 0;
    std::vector<int> h_part, h_nch;
    for (size_t i = 0; i < lat.size(); ++i) {
      const Geom& g = lat[i]->g;
      const int nch = (g.V + WG - 1) / WG;
      for (int r = 0; r < nrhs[i]; ++r) {
        h_part.push_back(total_chunks + r * nch);
        h_nch.push_back(nch);
      }
      nsys += nrhs[i];
      sites_rhs += (long long)nrhs[i] * g.V;
      total_chunks += nrhs[i] * nch;
      max_bvol = std::max(max_bvol, g.bvol);
    }
    uniform_bvol = lat[0]->g.bvol;
    for (auto* c : lat)
      if (c->g.bvol != uniform_bvol) uniform_bvol = 0;
    sys_part.ensure(sizeof(int) * nsys);
    sys_nchunks.ensure(sizeof(int) * nsys);
    HIPCK(hipMemcpy(sys_part.p, h_part.data(), sizeof(int) * nsys, hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(sys_nchunks.p, h_nch.data(), sizeof(int) * nsys, hipMemcpyHostToDevice));
    partials.ensure(sizeof(double) * (size_t)total_chunks * pw);
  }

  const LatDesc* lats(int prec, hipStream_t st, bool eo = false) {
    bool stale = !have_lats[prec] || (eo && !lats_eo[prec]);
    for (auto* c : lat) stale |= !c->have_links[prec] || !c->have_clov[prec];
    if (!stale) return d_lats[prec].as<LatDesc>();
    eo = eo || lats_eo[prec];
    h_lats[prec].clear();
    long long foff = 0;
    int sys0 = 0, part0 = 0;
    for (size_t i = 0; i < lat.size(); ++i) {
      wc_ctx* c = lat[i];
      ensure_links(c, prec, st);
      ensure_clover(c, prec, st);
      LatDesc L;
      L.g = c->g;
      L.gauge = c->links[prec].p;
      L.gscale = c->lscale[prec].as<float>();
      L.clov = c->clov[prec].p;
      L.cscale = c->cscale[prec].as<float>();
      L.foff = foff;
      L.nrhs = nrhs[i];
      L.sys0 = sys0;
      L.part0 = part0;
      L.nchunks = (c->g.V + WG - 1) / WG;
      L.tiles[0] = c->tiles[0].as<int>();
      L.tiles[1] = c->tiles[1].as<int>();
      L.clov_eo = nullptr;
      L.cscale_eo = nullptr;
      L.eo_sites = c->eo_sites.as<short>();
      L.eo_slot = c->eo_slot.as<short>();
      if (eo) {
        ensure_clover_eo(c, prec, st);
        L.clov_eo = c->clov_eo[prec].p;
        L.cscale_eo = c->cscale_eo[prec].as<float>();
      }
      h_lats[prec].push_back(L);
      foff += (long long)nrhs[i] * c->g.V;
      sys0 += nrhs[i];
      part0 += nrhs[i] * L.nchunks;
    }
    d_lats[prec].ensure(sizeof(LatDesc) * lat.size());
    HIPCK(hipMemcpy(d_lats[prec].p, h_lats[prec].data(), sizeof(LatDesc) * lat.size(), hipMemcpyHostToDevice));
    have_lats[prec] = true;
    lats_eo[prec] = eo;
    return d_lats[prec].as<LatDesc>();
  }

  // D_w items of rhs tile nr over the lattices selected by sel: 0 every lattice, 1 those
  // with 256-site blocks (whose chunks are blocks, so a launch may stage them), 2 the others
  const ItemList& items_dirac(int nr, int sel = 0) {
    const int key = 4 * nr + sel;
    auto it = dirac_items.find(key);
    if (it != dirac_items.end()) return it->second;
    // chunk-major: the items of one chunk's rhs tiles are consecutive, so one XCD runs them
    // at about the same time and its L2 serves the chunk's links and clover blocks to all
    // of them after one read from memory
    std::vector<WorkItem> v;
    for (size_t i = 0; i < lat.size(); ++i) {
      if ((sel == 1 && lat[i]->g.bvol != 256) || (sel == 2 && lat[i]->g.bvol == 256)) continue;
      const int nch = (lat[i]->g.V + WG - 1) / WG;
      for (int c = 0; c < nch; ++c)
        for (int r0 = 0; r0 < nrhs[i]; r0 += nr) v.push_back(WorkItem{(int)i, c, r0, std::min(nr, nrhs[i] - r0)});
    }
    ItemList& L = dirac_items[key];
    L.d.ensure(sizeof(WorkItem) * v.size());
    HIPCK(hipMemcpy(L.d.p, v.data(), sizeof(WorkItem) * v.size(), hipMemcpyHostToDevice));
    L.n = (int)v.size();
    return L;
  }

  // the block volumes of the batch, largest first
  std::vector<int> bvols() const {
    std::vector<int> v;
    for (auto* c : lat)
      if (std::find(v.begin(), v.end(), c->g.bvol) == v.end()) v.push_back(c->g.bvol);
    std::sort(v.rbegin(), v.rend());
    return v;
  }

  // block-solver items of the lattices with block volume bvol (0: every lattice)
  const ItemList& items_sap(int colour, int nr, int bvol = 0) {
    const int key = nr * 65536 + bvol;
    auto it = sap_items[colour].find(key);
    if (it != sap_items[colour].end()) return it->second;
    std::vector<WorkItem> v;
    for (size_t i = 0; i < lat.size(); ++i) {
      if (bvol && lat[i]->g.bvol != bvol) continue;
      const int nt = lat[i]->g.ntiles / 2;
      for (int t = 0; t < nt; ++t)
        for (int r0 = 0; r0 < nrhs[i]; r0 += nr) v.push_back(WorkItem{(int)i, t, r0, std::min(nr, nrhs[i] - r0)});
    }
    ItemList& L = sap_items[colour][key];
    L.d.ensure(sizeof(WorkItem) * v.size());
    HIPCK(hipMemcpy(L.d.p, v.data(), sizeof(WorkItem) * v.size(), hipMemcpyHostToDevice));
    L.n = (int)v.size();
    return L;
  }

  int sap_threads() const { return ((max_bvol + 63) / 64) * 64; }
};

static Batch& ctx_batch(wc_ctx* c, int nrhs) {
  auto it = c->batches.find(nrhs);
  if (it != c->batches.end()) return *it->second;
  auto b = std::make_unique<Batch>();
  b->init({c}, {nrhs});
  Batch& ref = *b;
  c->batches[nrhs] = std::move(b);
  return ref;
}

// Batches over several lattices, kept like the single-lattice ones (fields, item lists and
// captured graphs survive between calls) and keyed by the lattices and their rhs counts.
// A map on the heap that is never freed: entries go when one of their contexts changes its
// layout or is destroyed, and whatever a program leaks is not freed after the runtime.
using MultiKey = std::pair<std::vector<wc_ctx*>, std::vector<int>>;
static std::map<MultiKey, std::unique_ptr<Batch>>& multi_batches() {
  static auto* m = new std::map<MultiKey, std::unique_ptr<Batch>>();
  return *m;
}

static Batch& multi_batch(const std::vector<wc_ctx*>& ctxs, const std::vector<int>& nrhs) {
  auto& m = multi_batches();
  MultiKey key{ctxs, nrhs};
  auto it = m.find(key);
  if (it != m.end()) return *it->second;
  auto b = std::make_unique<Batch>();
  b->init(ctxs, nrhs);
  Batch& ref = *b;
  m[key] = std::move(b);
  return ref;
}

static void drop_multi_batches(wc_ctx* c) {
  auto& m = multi_batches();
  for (auto it = m.begin(); it != m.end();) {
    const auto& cs = it->first.first;
    if (std::find(cs.begin(), cs.end(), c) != cs.end())
      it = m.erase(it);
    else
      ++it;
  }
}

static void invalidate_batches(wc_ctx* c) {
  c->batches.clear();
  drop_multi_batches(c);
}

static int default_nr(int nrhs, int prec, bool sap, int eo) {
  if (nrhs <= 1) return 1;
  // even/odd block solver: each lane holds two sites, one rhs per work-group
  if (sap && eo) return 1;
  // 16-bit storage: two rhs share the block operator staged in LDS (4^4 blocks)
  if (sap) return is16(prec) ? 2 : 1;
  // FP64 with four rhs per lane spills; two fit in the register file
  if (prec == P_F64) return 2;
  return nrhs >= 4 ? 4 : nrhs;
}

static int pick_nr(wc_ctx* c, int nrhs, int prec, bool sap, int requested, int eo = 0) {
  int nr = requested > 0 ? requested : (sap ? (eo ? c->nr_sap_eo[prec] : c->nr_sap[prec]) : c->nr_dirac[prec]);
  if (nr <= 0) nr = default_nr(nrhs, prec, sap, eo);
  nr = std::min(nr, 4);
  // block-solver tiles keep the LDS exchange buffer within 64 KB: FP64 one rhs, else two
  if (sap) nr = std::min(nr, prec == P_F64 ? 1 : 2);
  return std::max(1, std::min(nr, std::max(1, nrhs)));
}

// ---------------------------------------------------------------------------- kernels on a batch

// Tile staging of the D_w input needs 256-site tiles in every lattice of the batch.  It
// pays for FP64 (whose spinors overflow L2 between the nine reads of each) and costs for
// FP32 / 16-bit (measured on MI355X); the WC_OPT_DIRAC_STAGE option of the batch's first
// context forces it off/on where allowed.
// Staging of a D_w launch: 0 none, 1 every item (all blocks have 256 sites), 2 split into
// a staged launch over the lattices with 256-site blocks and an unstaged one over the rest
static int dirac_stage_mode(const Batch& B, int prec, int nr) {
  // staged by default in every precision: at 24^3 x 48 and 32^3 x 64 staging is 3-15 %
  // faster for every storage; only where the whole problem sits in the Infinity Cache
  // (16^3 x 32) is it within a few per cent either way
  const int forced = B.lat[0]->opt_dirac_stage;
  const bool want = forced >= 0 ? forced != 0 : true;
  if (!want || dirac_stage_lds_bytes(prec, nr) > LDS_MAX_BYTES) return 0;
  if (B.uniform_bvol == 256) return 1;
  for (auto* c : B.lat)
    if (c->g.bvol == 256) return 2;
  return 0;
}

static void run_dirac(Batch& B, int prec, int nr, const Field& in, Field& out, const Field* y, double* partials,
                      const int* skip, int dagger, int block, hipStream_t st, const int* dead = nullptr) {
  const LatDesc* L = B.lats(prec, st);
  DiracLaunch a;
  a.lats = L;
  a.in = in.data();
  a.in_sc = in.scale();
  a.in_prec = in.prec;
  a.out = out.data();
  a.out_sc = out.scale();
  a.y = y ? y->data() : nullptr;
  a.y_sc = y ? y->scale() : nullptr;
  a.partials = partials;
  a.pw = B.pw;
  a.skip = skip;
  a.dagger = dagger;
  a.block = block;
  a.dead = dead;
  // (a tile of nr rhs that does not fit a work-group's LDS runs unstaged)
  const int mode = dirac_stage_mode(B, prec, nr);
  for (int sel : (mode == 2 ? std::array<int, 2>{1, 2} : std::array<int, 2>{0, -1})) {
    if (sel < 0) break;
    const ItemList& it = B.items_dirac(nr, sel);
    if (it.n == 0) continue;
    a.items = it.d.as<WorkItem>();
    a.nitems = it.n;
    a.stage = (mode == 1 || sel == 1) ? 1 : 0;
    launch_dirac(prec, nr, a, persistent_grid(it.n, 8), st);
  }
}

// Register caching of the block operator pays when the launch has about one work-group
// per CU (then nothing else could hide the reload latency); the WC_OPT_SAP_CACHE option of
// the batch's first context forces it on or off.
static int sap_cache_mode(const Batch& B, int nitems) {
  const int forced = B.lat[0]->opt_sap_cache;
  if (forced >= 0) return forced;
  return nitems <= 2 * device_cus() ? 1 : 0;
}


// odd_rho: residual on odd sites for the even/odd solver (see SapLaunch::odd_rho)
static void run_sap_halfsweep(Batch& B, int prec, int nr, int colour, int nmr, Field& rho, Field& z, Field& psi,
                              const int* skip, int first, int border, int wrho, int wz, int eo, hipStream_t st,
                              int odd_rho = 0) {
  require(nr >= 1 && nr <= (prec == P_F64 ? 1 : 2), WC_ERR_ARG, "block-solver rhs tile out of range");
  require((eo ? sap_eo_lds_bytes(prec, nr, B.max_bvol, 0) : sap_lds_bytes(prec, nr, B.sap_threads())) <= 65536,
          WC_ERR_GEOMETRY, "block too large for LDS");
  const LatDesc* L = B.lats(prec, st, eo != 0);
  // one launch per block volume of the batch, each with work-groups sized for its own
  // blocks (one launch sized for the largest would leave the lanes of smaller blocks idle)
  for (int bv : B.bvols()) {
    // the even/odd solver's border update runs from LDS entries when they fit a
    // work-group's LDS next to the exchange rows (else per site)
    int bentries = 0;
    for (auto* c : B.lat)
      if (c->g.bvol == bv) bentries = std::max(bentries, border_entry_count(c->g.B));
    if (eo && sap_eo_lds_bytes(prec, nr, bv, bentries) > LDS_MAX_BYTES) bentries = 0;
    const ItemList& it = B.items_sap(colour, nr, bv);
    if (it.n == 0) continue;
    SapLaunch a;
    a.lats = L;
    a.items = it.d.as<WorkItem>();
    a.nitems = it.n;
    a.colour = colour;
    a.nmr = nmr;
    a.rho = rho.data();
    a.rho_sc = rho.scale();
    a.z = z.data();
    a.z_sc = z.scale();
    a.psi = psi.data();
    a.psi_sc = psi.scale();
    a.skip = skip;
    a.first = first;
    a.border = border;
    a.write_rho = wrho;
    a.write_z = wz;
    a.cache = sap_cache_mode(B, it.n);
    a.uniform_bvol = bv;
    a.odd_rho = odd_rho;
    // (with the operator cached the launch has one work-group per CU, and the entries'
    // extra barrier costs more than the divergent per-site update: measured at 16^3 x 32)
    a.border_entries = (eo && !a.cache) ? bentries : 0;
    a.eo_rows = 2 * ((bv + 1) / 2);
    if (eo)
      launch_sap_eo(prec, nr, a, persistent_grid(it.n, 4), bv, st);
    else if (is16(prec) && nr == 2 && bv == 256)
      launch_sap_mr_lds(prec, nr, a, persistent_grid(it.n, 1), st);
    else
      launch_sap_mr(prec, nr, a, persistent_grid(it.n, 4), ((bv + 63) / 64) * 64, st);
  }
}

// ncy Schwarz cycles on rho (source), accumulating psi
static void run_sap(Batch& B, int prec, int nr, int ncy, int nmr, Field& rho, Field& z, Field& psi, const int* skip,
                    int eo, hipStream_t st) {
  for (int cy = 0; cy < ncy; ++cy)
    for (int c = 0; c < 2; ++c) {
      const bool last = (cy == ncy - 1);
      // the SAP's residual field is private: odd sites are read from it only on the first
      // visit of a block (later they hold the zero the previous solve left) and never stored
      run_sap_halfsweep(B, prec, nr, c, nmr, rho, z, psi, skip, cy == 0, !(cy == 0 && c == 0), !last,
                        !(last && c == 1), eo, st, cy == 0 ? 1 : 2);
    }
}

// pack / unpack canonical arrays of every lattice of the batch
static void pack_batch(Batch& B, int prec, const void* const* canon, Field& f, hipStream_t st) {
  long long off = 0;
  for (size_t i = 0; i < B.lat.size(); ++i) {
    const Geom& g = B.lat[i]->g;
    launch_pack_spinor(prec, g, B.nrhs[i], canon[i], (char*)f.data() + off * spinor_site_bytes(prec),
                       f.scale() ? f.scale() + off : nullptr, st);
    off += (long long)B.nrhs[i] * g.V;
  }
}
static void unpack_batch(Batch& B, int prec, const Field& f, void* const* canon, int colour_only, hipStream_t st) {
  long long off = 0;
  for (size_t i = 0; i < B.lat.size(); ++i) {
    const Geom& g = B.lat[i]->g;
    launch_unpack_spinor(prec, g, B.nrhs[i], (const char*)f.data() + off * spinor_site_bytes(prec),
                         f.scale() ? f.scale() + off : nullptr, canon[i], colour_only, st);
    off += (long long)B.nrhs[i] * g.V;
  }
}

// ---------------------------------------------------------------------------- FGCR

struct SolveSetup {
  int nkv, ncy, nmr, sap_prec, nr_d, nr_s, maxit, eo, stag, timing;
  int basis_prec;  // FGCR Krylov basis storage: P_F64 or P_F32 (then D phi_k in FP32 arithmetic)
  int nr_d32;      // rhs per lane of that FP32 D
  double tol;
  double drop2;    // squared per-cycle drop of the recursive residual (0: none)
};

// Events recorded between the phases of an eagerly launched restart cycle (solver
// parameter `timing`): the time between two marks is charged to the phase that ends at
// the later one.
enum Phase { PH_SAP = 0, PH_DIRAC = 1, PH_BLAS = 2 };
struct PhaseTimer {
  std::vector<hipEvent_t> ev;
  std::vector<int> tag;
  size_t n = 0;
  double t[3] = {0.0, 0.0, 0.0};
  PhaseTimer() = default;
  PhaseTimer(const PhaseTimer&) = delete;
  PhaseTimer& operator=(const PhaseTimer&) = delete;
  ~PhaseTimer() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  void mark(int phase, hipStream_t st) {
    if (n == ev.size()) {
      hipEvent_t e;
      HIPCK(hipEventCreate(&e));
      ev.push_back(e);
      tag.push_back(0);
    }
    tag[n] = phase;
    HIPCK(hipEventRecord(ev[n], st));
    ++n;
  }
  // after the stream has reached the last mark
  void collect() {
    for (size_t i = 1; i < n; ++i) {
      float ms = 0.f;
      HIPCK(hipEventElapsedTime(&ms, ev[i - 1], ev[i]));
      t[tag[i]] += ms;
    }
    n = 0;
  }
};
static void mark(PhaseTimer* tm, int phase, hipStream_t st) {
  if (tm) tm->mark(phase, st);
}

static VecLaunch vec_launch(Batch& B, const SolveSetup& s, hipStream_t st) {
  VecLaunch a;
  a.lats = B.lats(P_F64, st);
  const ItemList& it = B.items_dirac(1);
  a.items = it.d.as<WorkItem>();
  a.nitems = it.n;
  a.sys = B.sys.as<SysState>();
  a.skip = B.skip.as<int>();
  a.partials = B.partials.as<double>();
  a.pw = B.pw;
  a.k = 0;
  a.maxit = s.maxit;
  a.tol = s.tol;
  a.stag = s.stag;
  a.hist = B.hist.as<double>();
  a.hist_max = HIST_MAX;
  a.r = B.r.d.as<double2>();
  a.x = B.x.d.as<double2>();
  a.chi = B.d_chi.as<double2* const>();
  a.phi = B.d_phi.as<double2* const>();
  a.sp = nullptr;
  a.sp_sc = nullptr;
  a.arn = nullptr;
  a.dir = B.d_dir.as<void* const>();
  a.dir_sc = B.d_dir_sc.as<float* const>();
  a.dir_prec = s.sap_prec;
  a.fuse_sap = 0;
  a.q = B.d_chi.as<void* const>();
  a.w = nullptr;
  a.rq = a.r;
  a.dead = B.dead.p ? B.dead.as<int>() : nullptr;
  a.drop2 = s.drop2;
  return a;
}

// fgcr: the directions live in the preconditioner's storage (dir) and the basis chi in
// s.basis_prec (with an F32 basis, D phi_k is formed in FP32 into a buffer of its own, w);
// FGMRES-DR keeps its preconditioned basis Z in FP64 (phi), which its deflated restarts
// recombine
static void prepare_solver(Batch& B, const SolveSetup& s, bool fgcr = true) {
  const long long n = B.sites_rhs;
  B.x.ensure(P_F64, n);
  B.b.ensure(P_F64, n);
  B.r.ensure(P_F64, n);
  std::vector<double2*> pc(NKV_MAX, nullptr), pp(NKV_MAX, nullptr);
  std::vector<void*> pd(NKV_MAX, nullptr);
  std::vector<float*> pds(NKV_MAX, nullptr);
  if (fgcr && s.basis_prec != P_F64) {
    B.w.ensure(P_F32, n);
    B.r32.ensure(P_F32, n);
  }
  for (int k = 0; k < s.nkv; ++k) {
    B.chi[k].ensure(fgcr ? s.basis_prec : P_F64, n);
    pc[k] = B.chi[k].d.as<double2>();
    if (fgcr) {
      B.dir[k].ensure(s.sap_prec, n);
      pd[k] = B.dir[k].data();
      pds[k] = B.dir[k].scale();
    } else {
      B.phi[k].ensure(P_F64, n);
      pp[k] = B.phi[k].d.as<double2>();
    }
  }
  B.d_chi.ensure(sizeof(double2*) * NKV_MAX);
  B.d_phi.ensure(sizeof(double2*) * NKV_MAX);
  B.d_dir.ensure(sizeof(void*) * NKV_MAX);
  B.d_dir_sc.ensure(sizeof(float*) * NKV_MAX);
  HIPCK(hipMemcpy(B.d_chi.p, pc.data(), sizeof(double2*) * NKV_MAX, hipMemcpyHostToDevice));
  HIPCK(hipMemcpy(B.d_phi.p, pp.data(), sizeof(double2*) * NKV_MAX, hipMemcpyHostToDevice));
  HIPCK(hipMemcpy(B.d_dir.p, pd.data(), sizeof(void*) * NKV_MAX, hipMemcpyHostToDevice));
  HIPCK(hipMemcpy(B.d_dir_sc.p, pds.data(), sizeof(float*) * NKV_MAX, hipMemcpyHostToDevice));
  B.sap_rho.ensure(s.sap_prec, n);
  B.sap_z.ensure(s.sap_prec, n);
  B.sap_psi.ensure(s.sap_prec, n);
  B.sys.ensure(sizeof(SysState) * B.nsys);
  B.skip.ensure(sizeof(int) * B.nsys);
  // the cycle-ended flag and counts start at zero (a solve that ended abnormally could have
  // left them set); cleared here, outside any captured cycle
  B.dead.ensure(3 * sizeof(int));
  HIPCK(hipMemset(B.dead.p, 0, 3 * sizeof(int)));
  B.hist.ensure(sizeof(double) * HIST_MAX * B.nsys);
  // everything a captured cycle touches must exist before capture starts
  B.lats(P_F64, nullptr);
  B.lats(s.sap_prec, nullptr, s.eo != 0);
  if (fgcr && s.basis_prec != P_F64) B.lats(P_F32, nullptr);
  for (int nr : {1, s.nr_d, s.nr_d32})
    for (int sel = 0; sel < 3; ++sel) B.items_dirac(nr, sel);
  for (int bv : B.bvols())
    for (int c = 0; c < 2; ++c) B.items_sap(c, s.nr_s, bv);
  HIPCK(hipDeviceSynchronize());
}

// one restart cycle: nkv FGCR iterations; systems whose skip flag is set sit out
static void enqueue_cycle(Batch& B, const SolveSetup& s, hipStream_t st, PhaseTimer* tm = nullptr) {
  VecLaunch va = vec_launch(B, s, st);
  const int gv = persistent_grid(va.nitems, 8);
  const int* skip = B.skip.as<int>();
  mark(tm, PH_BLAS, st);
  const bool f64_basis = s.basis_prec == P_F64;
  // the recursion's residual: r itself with an FP64 basis; with an F32 one, an F32 copy that
  // the cycle's first conversion writes from the FP64 true residual
  va.rq = f64_basis ? B.r.data() : B.r32.data();
  for (int k = 0; k < s.nkv; ++k) {
    va.k = k;
    // the direction D phi_k: chi_k itself with an FP64 basis, else the F32 buffer w from
    // which Gram-Schmidt writes the F32 chi_k
    Field& wk = f64_basis ? B.chi[k] : B.w;
    va.w = wk.data();
    // phi_k = M_SAP(r / |r_k|) as the preconditioner stores it (the input of step k > 0 was
    // written by step k - 1's residual update)
    if (k == 0) {
      VecLaunch vs = va;
      vs.sp = B.sap_rho.data();
      vs.sp_sc = B.sap_rho.scale();
      launch_to_sap(s.sap_prec, s.basis_prec, vs, gv, st);
    }
    const int* dead = va.dead;
    run_sap(B, s.sap_prec, s.nr_s, s.ncy, s.nmr, B.sap_rho, B.sap_z, B.dir[k], skip, s.eo, st);
    mark(tm, PH_SAP, st);
    // w = D phi_k: FP64 arithmetic with an FP64 basis, FP32 (the single-precision
    // recursion) with an F32 one
    if (f64_basis)
      run_dirac(B, P_F64, s.nr_d, B.dir[k], wk, nullptr, nullptr, skip, 0, 0, st, dead);
    else
      run_dirac(B, P_F32, s.nr_d32, B.dir[k], wk, nullptr, nullptr, skip, 0, 0, st, dead);
    mark(tm, PH_DIRAC, st);
    // classical Gram-Schmidt: all inner products, then the update of chi_k and r (and the
    // next preconditioner input); a system whose first pass cancelled takes a second pass
    // (RED_GS2, k_gs_update2)
    VecLaunch vu = va;
    vu.sp = B.sap_rho.data();
    vu.sp_sc = B.sap_rho.scale();
    vu.fuse_sap = k + 1 < s.nkv;
    launch_gs_dots(s.basis_prec, va, gv, st);
    launch_reduce(RED_GS, va, B.nsys, B.sys_part.as<int>(), B.sys_nchunks.as<int>(), st);
    launch_gs_update(s.sap_prec, s.basis_prec, vu, gv, st);
    launch_reduce(RED_GS2, va, B.nsys, B.sys_part.as<int>(), B.sys_nchunks.as<int>(), st);
    launch_gs_update2(s.sap_prec, s.basis_prec, vu, gv, st);
    launch_reduce(RED_RNORM, va, B.nsys, B.sys_part.as<int>(), B.sys_nchunks.as<int>(), st);
    mark(tm, PH_BLAS, st);
  }
  // x += sum alpha phi; r = b - D x in FP64
  launch_backsub(va, B.nsys, st);
  launch_x_update_dir(va, gv, st);
  mark(tm, PH_BLAS, st);
  run_dirac(B, P_F64, s.nr_d, B.x, B.r, &B.b, B.partials.as<double>(), nullptr, 0, 0, st);
  mark(tm, PH_DIRAC, st);
  launch_reduce(RED_TRUE, va, B.nsys, B.sys_part.as<int>(), B.sys_nchunks.as<int>(), st);
  mark(tm, PH_BLAS, st);
}

static std::string setup_key(const SolveSetup& s) {
  char buf[240];
  snprintf(buf, sizeof buf, "%d/%d/%d/%d/%d/%d/%d/%d/%d/%.17g/%d/%.17g/%d", s.nkv, s.ncy, s.nmr, s.sap_prec,
           s.nr_d, s.nr_s, s.maxit, s.eo, s.stag, s.tol, s.basis_prec, s.drop2, s.nr_d32);
  return buf;
}

// Key of a captured cycle: the set-up, the kernel-selecting options and the device address
// of every buffer the cycle's launches name.  A field that another call reallocated (a
// wider precision asked of the batch's Schwarz fields, for instance) changes the key, so
// a graph is never replayed over memory that was freed.
static std::string graph_key(const Batch& B, const SolveSetup& s) {
  std::string k = setup_key(s);
  char buf[40];
  auto add = [&](const void* q) {
    snprintf(buf, sizeof buf, "|%p", q);
    k += buf;
  };
  add(B.x.data());
  add(B.b.data());
  add(B.r.data());
  add(B.w.data());
  add(B.r32.data());
  for (int i = 0; i < s.nkv; ++i) {
    add(B.chi[i].data());
    add(B.phi[i].data());
    add(B.dir[i].data());
    add(B.dir[i].scale());
  }
  add(B.d_dir.p);
  add(B.d_dir_sc.p);
  for (const Field* f : {&B.sap_rho, &B.sap_z, &B.sap_psi}) {
    add(f->data());
    add(f->scale());
  }
  for (const DevBuf* d : {&B.dead, &B.sys, &B.skip, &B.partials, &B.hist, &B.d_chi, &B.d_phi, &B.d_arn_v, &B.arn,
                          &B.sys_part, &B.sys_nchunks, &B.d_lats[P_F64], &B.d_lats[s.sap_prec], &B.d_lats[P_F32]})
    add(d->p);
  add(B.arn_vlast.data());
  for (const auto& kv : B.dirac_items) add(kv.second.d.p);
  for (int c = 0; c < 2; ++c)
    for (const auto& kv : B.sap_items[c]) add(kv.second.d.p);
  k += "|" + std::to_string(B.lat[0]->opt_sap_cache) + "," + std::to_string(B.lat[0]->opt_dirac_stage);
  return k;
}

// what the host reads back of each system after a solve
static void fill_stats(Batch& B, const std::vector<SysState>& hs, float ms, const double* tph,
                       std::vector<wc_solver_stats>& stats, int* rc_out) {
  std::vector<double> hist((size_t)HIST_MAX * B.nsys);
  HIPCK(hipMemcpy(hist.data(), B.hist.p, sizeof(double) * hist.size(), hipMemcpyDeviceToHost));
  int rc = WC_OK;
  stats.resize(B.nsys);
  for (int i = 0; i < B.nsys; ++i) {
    wc_solver_stats& o = stats[i];
    std::memset(&o, 0, sizeof o);
    const SysState& S = hs[i];
    o.iters = S.iters;
    o.restarts = S.restarts;
    o.breakdown = S.breakdown;
    o.reorth = S.reorths;
    o.stagnated = S.stagnated;
    o.rel_true_res = S.bnorm2 > 0 ? std::sqrt(S.rnorm2 / S.bnorm2) : 0.0;
    o.time_ms = ms;
    o.nhist = std::min(S.restarts, HIST_MAX);
    for (int h = 0; h < o.nhist; ++h) o.res_hist[h] = hist[(size_t)i * HIST_MAX + h];
    o.timed = tph ? 1 : 0;
    if (tph) {
      o.t_setup_ms = tph[3];
      o.t_cycles_ms = tph[4];
      o.t_finish_ms = tph[5];
      o.t_sap_ms = tph[PH_SAP];
      o.t_dirac_ms = tph[PH_DIRAC];
      o.t_blas_ms = tph[PH_BLAS];
    }
    if (S.breakdown)
      o.status = WC_ERR_BREAKDOWN;
    else if (S.bnorm2 > 0 && !(S.rnorm2 <= S.tol2))
      o.status = WC_ERR_NOT_CONVERGED;
    else
      o.status = WC_OK;
    if (rc == WC_OK && o.status != WC_OK) rc = o.status;
  }
  *rc_out = rc;
}

static int fgcr_solve(Batch& B, const SolveSetup& s, bool x0_given, bool use_graph, wc_ctx* cap_owner,
                      std::vector<wc_solver_stats>& stats, hipStream_t st) {
  HipEvent e0, e1, e_setup, e_cycles;
  std::unique_ptr<PhaseTimer> tm(s.timing ? new PhaseTimer : nullptr);
  if (tm) use_graph = false;
  HIPCK(hipEventRecord(e0, st));
  VecLaunch va = vec_launch(B, s, st);
  const int gv = persistent_grid(va.nitems, 8);
  // |b|^2 -> tolerance; r = b (x = 0) or r = b - D x0
  launch_norm2(va, B.b.d.as<double2>(), gv, st);
  launch_reduce(RED_BNORM, va, B.nsys, B.sys_part.as<int>(), B.sys_nchunks.as<int>(), st);
  if (x0_given) {
    launch_zero_if_b0(va, B.x.d.as<double2>(), gv, st);
    run_dirac(B, P_F64, s.nr_d, B.x, B.r, &B.b, B.partials.as<double>(), nullptr, 0, 0, st);
    launch_reduce(RED_INITR, va, B.nsys, B.sys_part.as<int>(), B.sys_nchunks.as<int>(), st);
  } else {
    HIPCK(hipMemsetAsync(B.x.data(), 0, spinor_bytes(P_F64, B.sites_rhs), st));
    launch_copy_f64(va, B.r.d.as<double2>(), B.b.d.as<double2>(), gv, st);
  }
  HIPCK(hipGetLastError());
  HIPCK(hipEventRecord(e_setup, st));

  hipGraphExec_t exec = nullptr;
  if (use_graph) {
    const std::string key = graph_key(B, s);
    if (B.graph && B.graph_key == key) {
      exec = B.graph;
    } else {
      if (B.graph) {
        HIPCK(hipGraphExecDestroy(B.graph));
        B.graph = nullptr;
      }
      if (!cap_owner->cap) HIPCK(hipStreamCreateWithFlags(&cap_owner->cap, hipStreamNonBlocking));
      B.graph = capture_graph(cap_owner->cap, [&](hipStream_t cs) { enqueue_cycle(B, s, cs); });
      B.graph_key = key;
      exec = B.graph;
    }
  }

  std::vector<int> h_skip(B.nsys);
  const int max_restarts = s.maxit + 1;
  for (int rs = 0; rs < max_restarts; ++rs) {
    HIPCK(hipMemcpyAsync(h_skip.data(), B.skip.p, sizeof(int) * B.nsys, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (tm) tm->collect();
    bool all = true;
    for (int v : h_skip) all &= (v != 0);
    if (all) break;
    if (exec)
      HIPCK(hipGraphLaunch(exec, st));
    else
      enqueue_cycle(B, s, st, tm.get());
    HIPCK(hipGetLastError());
  }
  HIPCK(hipEventRecord(e_cycles, st));
  HIPCK(hipEventRecord(e1, st));
  HIPCK(hipEventSynchronize(e1));
  float ms = 0.f, ms_setup = 0.f, ms_cycles = 0.f;
  HIPCK(hipEventElapsedTime(&ms, e0, e1));
  HIPCK(hipEventElapsedTime(&ms_setup, e0, e_setup));
  HIPCK(hipEventElapsedTime(&ms_cycles, e_setup, e_cycles));
  double tph[6] = {0, 0, 0, ms_setup, ms_cycles, 0};
  if (tm)
    for (int q = 0; q < 3; ++q) tph[q] = tm->t[q];

  std::vector<SysState> hs(B.nsys);
  HIPCK(hipMemcpy(hs.data(), B.sys.p, sizeof(SysState) * B.nsys, hipMemcpyDeviceToHost));
  int rc = WC_OK;
  fill_stats(B, hs, ms, tm ? tph : nullptr, stats, &rc);
  return rc;
}

static SolveSetup make_setup(const wc_solver_params& p, wc_ctx* c, int max_nrhs) {
  require(p.nkv >= 1 && p.nkv <= NKV_MAX, WC_ERR_ARG, "nkv must be in 1..32");
  require(p.ncy >= 1 && p.nmr >= 1, WC_ERR_ARG, "ncy and nmr must be >= 1");
  require(p.sap_prec >= 0 && p.sap_prec <= 3, WC_ERR_ARG, "bad sap_prec");
  require(p.tol > 0 && p.maxit >= 1, WC_ERR_ARG, "tol must be > 0 and maxit >= 1");
  require(p.eo == 0 || p.eo == 1, WC_ERR_ARG, "eo must be 0 or 1");
  require(p.dagger == 0 || p.dagger == 1, WC_ERR_ARG, "dagger must be 0 or 1");
  require(p.stag >= 0, WC_ERR_ARG, "stag must be >= 0");
  require(p.timing == 0 || p.timing == 1, WC_ERR_ARG, "timing must be 0 or 1");
  require(p.basis_prec == WC_F64 || p.basis_prec == WC_F32, WC_ERR_ARG, "basis_prec must be WC_F64 or WC_F32");
  require(p.drop >= 0.0 && p.drop < 1.0, WC_ERR_ARG, "drop must be in [0, 1)");
  SolveSetup s;
  s.basis_prec = p.basis_prec;
  // drop 0: none with an FP64 basis; 1e-6 with an F32 one, whose stored vectors leave the
  // recursive residual a few 1e-8 of the cycle's starting residual from the true one
  const double drop = p.drop > 0.0 ? p.drop : (p.basis_prec == WC_F32 ? 1e-6 : 0.0);
  s.drop2 = drop * drop;
  s.nkv = p.nkv;
  s.ncy = p.ncy;
  s.nmr = p.nmr;
  s.sap_prec = p.sap_prec;
  s.tol = p.tol;
  s.maxit = p.maxit;
  s.eo = p.eo ? 1 : 0;
  s.stag = p.stag;
  s.timing = p.timing;
  s.nr_d = pick_nr(c, max_nrhs, P_F64, false, p.nr_dirac);
  s.nr_d32 = pick_nr(c, max_nrhs, P_F32, false, 0);
  s.nr_s = pick_nr(c, max_nrhs, p.sap_prec, true, p.nr_sap, s.eo);
  return s;
}

// ---------------------------------------------------------------------------- FGMRES-DR

static VecLaunch arn_launch(Batch& B, const SolveSetup& s, hipStream_t st) {
  VecLaunch a = vec_launch(B, s, st);
  a.chi = B.d_arn_v.as<double2* const>();
  a.arn = B.arn.as<ArnState>();
  a.dead = nullptr;
  return a;
}

static void prepare_fgmres(Batch& B, const SolveSetup& s) {
  prepare_solver(B, s, false);
  B.arn_vlast.ensure(P_F64, B.sites_rhs);
  std::vector<double2*> pv(NKV_MAX + 1, nullptr);
  for (int k = 0; k < s.nkv; ++k) pv[k] = B.chi[k].d.as<double2>();
  pv[s.nkv] = B.arn_vlast.d.as<double2>();
  B.d_arn_v.ensure(sizeof(double2*) * (NKV_MAX + 1));
  HIPCK(hipMemcpy(B.d_arn_v.p, pv.data(), sizeof(double2*) * (NKV_MAX + 1), hipMemcpyHostToDevice));
  B.arn.ensure(sizeof(ArnState) * B.nsys);
}

// Arnoldi columns j0 .. m-1 of one cycle; systems whose cycle ended sit out
static void enqueue_arn_cycle(Batch& B, const SolveSetup& s, int j0, hipStream_t st) {
  VecLaunch va = arn_launch(B, s, st);
  const int gv = persistent_grid(va.nitems, 8);
  const int* skip = B.skip.as<int>();
  for (int j = j0; j < s.nkv; ++j) {
    va.k = j;
    VecLaunch vs = va;
    vs.sp = B.sap_rho.data();
    vs.sp_sc = B.sap_rho.scale();
    launch_arn_to_sap(s.sap_prec, vs, gv, st);
    run_sap(B, s.sap_prec, s.nr_s, s.ncy, s.nmr, B.sap_rho, B.sap_z, B.sap_psi, skip, s.eo, st);
    vs.sp = B.sap_psi.data();
    vs.sp_sc = B.sap_psi.scale();
    launch_arn_from_sap(s.sap_prec, vs, gv, st);
    Field& next = (j + 1 < s.nkv) ? B.chi[j + 1] : B.arn_vlast;
    run_dirac(B, P_F64, s.nr_d, B.phi[j], next, nullptr, nullptr, skip, 0, 0, st);
    launch_arn_dots(va, gv, st);
    launch_arn_reduce(1, va, B.nsys, B.sys_part.as<int>(), B.sys_nchunks.as<int>(), s.nkv, st);
    launch_arn_update1(va, gv, st);
    launch_arn_reduce(2, va, B.nsys, B.sys_part.as<int>(), B.sys_nchunks.as<int>(), s.nkv, st);
    launch_arn_update(va, gv, st);
  }
}

// The deflated restart of one system on the host: P from the k harmonic Ritz vectors of
// smallest |theta| and the least-squares residual s, the new (k+1) x k matrix P^H Hbar P_k,
// its Givens factorisation and the new residual coefficients.  Returns false when the
// small problem is singular (the caller then restarts without deflation).
static bool deflate_host(int mm, int k, ArnState& A, const std::vector<dense::cd>& sres, std::vector<dense::cd>& cnew) {
  using dense::cd;
  const int ld = ARN_LD;
  std::vector<cd> H((size_t)ld * NKV_MAX);
  for (int j = 0; j < mm; ++j)
    for (int i = 0; i <= mm; ++i) H[i + j * ld] = cd(A.H[i + j * ld].x, A.H[i + j * ld].y);
  std::vector<cd> theta(mm), G((size_t)mm * mm);
  if (!dense::harmonic_ritz(mm, H.data(), ld, theta.data(), G.data(), mm)) return false;
  std::vector<cd> P((size_t)ld * ld, cd(0.0));
  for (int l = 0; l < k; ++l)
    for (int i = 0; i < mm; ++i) P[i + l * ld] = G[i + l * mm];
  for (int i = 0; i <= mm; ++i) P[i + k * ld] = sres[i];
  if (!dense::orthonormalise(mm + 1, k + 1, P.data(), ld)) return false;
  // Hn = P^H Hbar P[:mm, :k] ; cnew = P^H s
  std::vector<cd> HP((size_t)ld * k, cd(0.0)), Hn((size_t)ld * k, cd(0.0));
  for (int l = 0; l < k; ++l)
    for (int i = 0; i <= mm; ++i) {
      cd t = 0.0;
      for (int j = 0; j < mm; ++j) t += H[i + j * ld] * P[j + l * ld];
      HP[i + l * ld] = t;
    }
  for (int l = 0; l < k; ++l)
    for (int r = 0; r <= k; ++r) {
      cd t = 0.0;
      for (int i = 0; i <= mm; ++i) t += std::conj(P[i + r * ld]) * HP[i + l * ld];
      Hn[r + l * ld] = t;
    }
  cnew.assign(k + 1, cd(0.0));
  for (int r = 0; r <= k; ++r) {
    cd t = 0.0;
    for (int i = 0; i <= mm; ++i) t += std::conj(P[i + r * ld]) * sres[i];
    cnew[r] = t;
  }
  // the device state of the next cycle: Hbar = Hn, its rotations and rotated coefficients
  std::vector<cd> R(Hn), g(cnew);
  g.resize(ld, cd(0.0));
  std::vector<dense::Rot> rots;
  dense::givens_qr(k + 1, k, R.data(), ld, g.data(), rots);
  if ((int)rots.size() > ARN_ROT_MAX - NKV_MAX - 1) return false;
  for (int i = 0; i < ld * NKV_MAX; ++i) A.H[i] = make_double2(0.0, 0.0);
  for (int l = 0; l < k; ++l)
    for (int r = 0; r <= k; ++r) A.H[r + l * ld] = make_double2(Hn[r + l * ld].real(), Hn[r + l * ld].imag());
  for (int i = 0; i < ld; ++i) A.g[i] = make_double2(g[i].real(), g[i].imag());
  A.nrot = (int)rots.size();
  for (int q = 0; q < A.nrot; ++q) {
    A.rc[q] = rots[q].c;
    A.rs[q] = make_double2(rots[q].s.real(), rots[q].s.imag());
    A.rp[q] = rots[q].p;
  }
  for (int i = 0; i < ld * ld; ++i) A.P[i] = make_double2(P[i].real(), P[i].imag());
  A.pin = mm + 1;
  A.pout = k + 1;
  A.lucky = 0;
  return true;
}

static int fgmres_dr_solve(Batch& B, const SolveSetup& s, int kdefl, bool x0_given, bool use_graph, wc_ctx* cap_owner,
                           std::vector<wc_solver_stats>& stats, hipStream_t st) {
  using dense::cd;
  HipEvent e0, e1;
  HIPCK(hipEventRecord(e0, st));
  VecLaunch va = arn_launch(B, s, st);
  const int gv = persistent_grid(va.nitems, 8);
  const int n = B.nsys, m = s.nkv, ld = ARN_LD;
  launch_norm2(va, B.b.d.as<double2>(), gv, st);
  launch_reduce(RED_BNORM, va, n, B.sys_part.as<int>(), B.sys_nchunks.as<int>(), st);
  if (x0_given) {
    launch_zero_if_b0(va, B.x.d.as<double2>(), gv, st);
    run_dirac(B, P_F64, s.nr_d, B.x, B.r, &B.b, B.partials.as<double>(), nullptr, 0, 0, st);
    launch_reduce(RED_INITR, va, n, B.sys_part.as<int>(), B.sys_nchunks.as<int>(), st);
  } else {
    HIPCK(hipMemsetAsync(B.x.data(), 0, spinor_bytes(P_F64, B.sites_rhs), st));
    launch_copy_f64(va, B.r.d.as<double2>(), B.b.d.as<double2>(), gv, st);
  }
  HIPCK(hipGetLastError());

  std::vector<SysState> hs(n);
  std::vector<ArnState> ha(n);
  std::vector<std::vector<cd>> cvec(n), sres(n);
  auto get_sys = [&] {
    HIPCK(hipMemcpyAsync(hs.data(), B.sys.p, sizeof(SysState) * n, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
  };
  auto put_arn = [&] {
    HIPCK(hipMemcpyAsync(B.arn.p, ha.data(), sizeof(ArnState) * n, hipMemcpyHostToDevice, st));
    HIPCK(hipStreamSynchronize(st));
  };
  int j0 = 0;
  for (int rs = 0; rs <= s.maxit; ++rs) {
    get_sys();
    bool all = true;
    for (const SysState& S : hs) all &= (S.converged != 0);
    if (all) break;
    if (j0 == 0) {
      // a cycle without deflation: V_0 = r / |r|, c = |r| e_0
      for (int i = 0; i < n; ++i) {
        ArnState& A = ha[i];
        A.nrot = 0;
        A.lucky = 0;
        A.pin = A.pout = 0;
        for (int q = 0; q < ld * NKV_MAX; ++q) A.H[q] = make_double2(0.0, 0.0);
        for (int q = 0; q < ld; ++q) A.g[q] = make_double2(0.0, 0.0);
        A.g[0] = make_double2(std::sqrt(hs[i].rnorm2), 0.0);
        cvec[i].assign(1, cd(std::sqrt(hs[i].rnorm2), 0.0));
      }
      put_arn();
      launch_arn_init(va, gv, st);
    }
    if (use_graph) {
      const std::string base = graph_key(B, s);
      if (base != B.arn_key) {
        // a buffer of the captured cycles moved: none of them may run again
        for (auto& kv : B.arn_graphs) HIPCK(hipGraphExecDestroy(kv.second));
        B.arn_graphs.clear();
        B.arn_key = base;
      }
      const std::string key = std::to_string(j0);
      auto it = B.arn_graphs.find(key);
      if (it == B.arn_graphs.end()) {
        if (!cap_owner->cap) HIPCK(hipStreamCreateWithFlags(&cap_owner->cap, hipStreamNonBlocking));
        HIPCK(hipStreamSynchronize(st));
        hipGraphExec_t exec =
            capture_graph(cap_owner->cap, [&](hipStream_t cs) { enqueue_arn_cycle(B, s, j0, cs); });
        it = B.arn_graphs.emplace(key, exec).first;
      }
      HIPCK(hipGraphLaunch(it->second, st));
    } else {
      enqueue_arn_cycle(B, s, j0, st);
    }
    HIPCK(hipGetLastError());
    HIPCK(hipMemcpyAsync(ha.data(), B.arn.p, sizeof(ArnState) * n, hipMemcpyDeviceToHost, st));
    get_sys();
    // least squares of every active system: x += Z d
    for (int i = 0; i < n; ++i) {
      SysState& S = hs[i];
      if (S.converged) continue;
      const int mm = S.k_done;
      std::vector<cd> H((size_t)ld * NKV_MAX), c(cvec[i]), d(std::max(mm, 1), cd(0.0));
      c.resize(mm + 1, cd(0.0));
      for (int j = 0; j < mm; ++j)
        for (int r = 0; r <= mm; ++r) H[r + j * ld] = cd(ha[i].H[r + j * ld].x, ha[i].H[r + j * ld].y);
      if (mm == 0 || S.breakdown || !dense::lstsq(mm + 1, mm, H.data(), ld, c.data(), d.data())) {
        S.breakdown = 1;
        d.assign(std::max(mm, 1), cd(0.0));
      }
      sres[i].assign(mm + 1, cd(0.0));
      for (int r = 0; r <= mm; ++r) {
        cd t = c[r];
        for (int j = 0; j < mm; ++j) t -= H[r + j * ld] * d[j];
        sres[i][r] = t;
      }
      for (int j = 0; j < mm; ++j) S.alpha[j] = make_double2(d[j].real(), d[j].imag());
    }
    HIPCK(hipMemcpyAsync(B.sys.p, hs.data(), sizeof(SysState) * n, hipMemcpyHostToDevice, st));
    HIPCK(hipStreamSynchronize(st));
    launch_x_update(va, gv, st);
    run_dirac(B, P_F64, s.nr_d, B.x, B.r, &B.b, B.partials.as<double>(), nullptr, 0, 0, st);
    launch_reduce(RED_TRUE, va, n, B.sys_part.as<int>(), B.sys_nchunks.as<int>(), st);
    HIPCK(hipGetLastError());
    std::vector<int> mm_of(n);
    for (int i = 0; i < n; ++i) mm_of[i] = hs[i].k_done;
    get_sys();
    // next cycle: deflated when every active system has k+1 columns to deflate from and its
    // recomputed residual still agrees with the cycle's least-squares residual (otherwise
    // the restart starts afresh from the true residual)
    bool defl = kdefl > 0;
    for (int i = 0; i < n; ++i) {
      if (hs[i].converged) continue;
      double sn = 0.0;
      for (const cd& z : sres[i]) sn += std::norm(z);
      defl = defl && mm_of[i] >= kdefl + 1 && !ha[i].lucky && hs[i].rnorm2 <= 100.0 * sn;
    }
    if (defl) {
      for (int i = 0; i < n && defl; ++i) {
        if (hs[i].converged) continue;
        std::vector<cd> cn;
        defl = deflate_host(mm_of[i], kdefl, ha[i], sres[i], cn);
        cvec[i] = cn;
      }
    }
    if (defl) {
      put_arn();
      launch_arn_recombine(va, gv, st);
      HIPCK(hipGetLastError());
      j0 = kdefl;
    } else {
      j0 = 0;
    }
  }
  HIPCK(hipEventRecord(e1, st));
  HIPCK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCK(hipEventElapsedTime(&ms, e0, e1));
  get_sys();
  int rc = WC_OK;
  fill_stats(B, hs, ms, nullptr, stats, &rc);
  return rc;
}

// ---------------------------------------------------------------------------- helpers for the C interface

static hipStream_t S(void* stream) { return (hipStream_t)stream; }

template <class F> static int guarded(F f) {
  try {
    f();
    return WC_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return WC_ERR_OOM;
  } catch (...) {
    g_last_error = "unexpected error";
    return WC_ERR_HIP;
  }
}

static void check_prec(int prec) { require(prec >= 0 && prec <= 3, WC_ERR_ARG, "bad precision"); }

static void layout(wc_ctx* c, const int* block, hipStream_t st) {
  require(valid_block(c->dims, block), WC_ERR_GEOMETRY,
          "block must divide the lattice into an even number of blocks along every axis, <= 256 sites");
  invalidate_batches(c);
  for (int m = 0; m < 4; ++m) c->block[m] = block[m];
  c->g = make_geom(c->dims, block, c->bc_t);
  std::vector<int> t0, t1;
  for (int t = 0; t < c->g.ntiles; ++t) {
    int tc[4];
    tile_coords(c->g, t, tc);
    (tile_colour(tc) ? t1 : t0).push_back(t);
  }
  c->tiles[0].ensure(sizeof(int) * t0.size());
  c->tiles[1].ensure(sizeof(int) * t1.size());
  HIPCK(hipMemcpy(c->tiles[0].p, t0.data(), sizeof(int) * t0.size(), hipMemcpyHostToDevice));
  HIPCK(hipMemcpy(c->tiles[1].p, t1.data(), sizeof(int) * t1.size(), hipMemcpyHostToDevice));
  // even and odd sites of a tile in local order, for both parities of the tile's corner
  const int nh = (c->g.bvol + 1) / 2;
  // and each site's slot when the even sites come first, then the odd ones, in that order
  std::vector<short> lut(4 * (size_t)nh, (short)-1), slot(2 * (size_t)c->g.bvol);
  for (int cp = 0; cp < 2; ++cp) {
    int cnt[2] = {0, 0};
    for (int l = 0; l < c->g.bvol; ++l) {
      int lc[4];
      local_coords(c->g, l, lc);
      const int par = (cp + lc[0] + lc[1] + lc[2] + lc[3]) & 1;
      slot[(size_t)cp * c->g.bvol + l] = (short)(par * nh + cnt[par]);
      lut[(size_t)(2 * cp + par) * nh + cnt[par]++] = (short)l;
    }
  }
  c->eo_sites.ensure(sizeof(short) * lut.size());
  HIPCK(hipMemcpy(c->eo_sites.p, lut.data(), sizeof(short) * lut.size(), hipMemcpyHostToDevice));
  c->eo_slot.ensure(sizeof(short) * slot.size());
  HIPCK(hipMemcpy(c->eo_slot.p, slot.data(), sizeof(short) * slot.size(), hipMemcpyHostToDevice));
  for (int p = 0; p < 4; ++p) {
    c->have_links[p] = false;
    c->have_clov[p] = false;
    c->have_clov_eo[p] = false;
  }
  ensure_links(c, P_F64, st);
  if (c->have_clover) {
    c->clov[P_F64].ensure((size_t)c->g.V * clover_site_bytes(P_F64));
    launch_clover_build(c->g, c->links[P_F64].p, c->m0, c->csw, c->clov[P_F64].p, st);
    HIPCK(hipGetLastError());
    c->have_clov[P_F64] = true;
  }
}

}  // namespace wc

wc_ctx::~wc_ctx() {
  batches.clear();
  wc::drop_multi_batches(this);
  if (cap) (void)hipStreamDestroy(cap);
}

using namespace wc;

extern "C" {

void wc_default_params(wc_solver_params* p) {
  if (!p) return;
  p->nkv = 16;
  p->ncy = 5;
  p->nmr = 4;
  p->sap_prec = WC_F32;
  p->tol = 1e-10;
  p->maxit = 10000;
  p->x0_given = 0;
  p->use_graph = 1;
  p->nr_dirac = 0;
  p->nr_sap = 0;
  p->eo = 0;
  p->dagger = 0;
  p->stag = 3;
  p->timing = 0;
  p->basis_prec = WC_F64;
  p->drop = 0.0;
}

int wc_set_option(wc_ctx* c, int option, int value) {
  return guarded([&] {
    require(c, WC_ERR_ARG, "null context");
    require(value >= -1 && value <= 1, WC_ERR_ARG, "option value must be -1, 0 or 1");
    if (option == WC_OPT_SAP_CACHE)
      c->opt_sap_cache = value;
    else if (option == WC_OPT_DIRAC_STAGE)
      c->opt_dirac_stage = value;
    else
      require(false, WC_ERR_ARG, "unknown option");
  });
}

int wc_set_tiles(wc_ctx* c, int prec, int nr_dirac, int nr_sap, int nr_sap_eo) {
  return guarded([&] {
    require(c, WC_ERR_ARG, "null context");
    check_prec(prec);
    const int smax = prec == P_F64 ? 1 : 2;
    require(nr_dirac >= 0 && nr_dirac <= 4, WC_ERR_ARG, "nr_dirac must be in 0..4");
    require(nr_sap >= 0 && nr_sap <= smax && nr_sap_eo >= 0 && nr_sap_eo <= smax, WC_ERR_ARG,
            "block-solver tiles must be in 0..2 (0..1 for FP64)");
    c->nr_dirac[prec] = nr_dirac;
    c->nr_sap[prec] = nr_sap;
    c->nr_sap_eo[prec] = nr_sap_eo;
  });
}

int wc_create_gauge(wc_ctx** ctx, const int dims[4], const int block[4], const void* U, int bc_t, void* stream) {
  return guarded([&] {
    require(ctx && dims && block && U, WC_ERR_ARG, "null argument");
    require(bc_t == 1 || bc_t == -1, WC_ERR_ARG, "bc_t must be +1 or -1");
    for (int m = 0; m < 4; ++m) require(dims[m] >= 2, WC_ERR_GEOMETRY, "lattice extents must be >= 2");
    auto c = std::make_unique<wc_ctx>();
    HIPCK(hipGetDevice(&c->dev));
    scratch_setup(c->dev);
    for (int m = 0; m < 4; ++m) c->dims[m] = dims[m];
    c->bc_t = bc_t;
    const long long V = (long long)dims[0] * dims[1] * dims[2] * dims[3];
    require(V < (1LL << 30), WC_ERR_GEOMETRY, "lattice too large");
    c->Ucanon.ensure((size_t)V * 4 * 9 * 16);
    HIPCK(hipMemcpyAsync(c->Ucanon.p, U, (size_t)V * 4 * 9 * 16, hipMemcpyDeviceToDevice, S(stream)));
    layout(c.get(), block, S(stream));
    HIPCK(hipStreamSynchronize(S(stream)));
    *ctx = c.release();
  });
}

int wc_create_clover(wc_ctx* c, double m0, double csw, void* stream) {
  return guarded([&] {
    require(c, WC_ERR_ARG, "null context");
    c->m0 = m0;
    c->csw = csw;
    c->clov[P_F64].ensure((size_t)c->g.V * clover_site_bytes(P_F64));
    launch_clover_build(c->g, c->links[P_F64].p, m0, csw, c->clov[P_F64].p, S(stream));
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(S(stream)));
    c->have_clover = true;
    for (int p = 0; p < 4; ++p) {
      c->have_clov[p] = (p == P_F64);
      c->have_clov_eo[p] = false;
    }
    for (auto& kv : c->batches)
      for (int p = 0; p < 4; ++p) kv.second->have_lats[p] = false;
    for (auto& kv : multi_batches()) {
      const auto& cs = kv.first.first;
      if (std::find(cs.begin(), cs.end(), c) != cs.end())
        for (int p = 0; p < 4; ++p) kv.second->have_lats[p] = false;
    }
  });
}

int wc_set_block(wc_ctx* c, const int block[4], void* stream) {
  return guarded([&] {
    require(c && block, WC_ERR_ARG, "null argument");
    layout(c, block, S(stream));
  });
}

int wc_clover_export(wc_ctx* c, void* A, void* stream) {
  return guarded([&] {
    require(c && A, WC_ERR_ARG, "null argument");
    require(c->have_clover, WC_ERR_STATE, "clover term not created");
    launch_clover_export(c->g, c->clov[P_F64].p, A, S(stream));
    HIPCK(hipGetLastError());
  });
}

int wc_apply_D(wc_ctx* c, void* out, const void* in, int nrhs, int prec, int region, int dagger, void* stream) {
  return guarded([&] {
    require(c && out && in && nrhs >= 1, WC_ERR_ARG, "null argument or nrhs < 1");
    check_prec(prec);
    require(region == WC_FULL || region == WC_BLOCKS, WC_ERR_ARG, "bad region");
    require(c->have_clover, WC_ERR_STATE, "clover term not created");
    hipStream_t st = S(stream);
    Batch& B = ctx_batch(c, nrhs);
    B.ain[prec].ensure(prec, B.sites_rhs);
    B.aout[prec].ensure(prec, B.sites_rhs);
    const void* ins[1] = {in};
    void* outs[1] = {out};
    pack_batch(B, prec, ins, B.ain[prec], st);
    run_dirac(B, prec, pick_nr(c, nrhs, prec, false, 0), B.ain[prec], B.aout[prec], nullptr, nullptr, nullptr,
              dagger ? 1 : 0, region == WC_BLOCKS, st);
    unpack_batch(B, prec, B.aout[prec], outs, -1, st);
    HIPCK(hipGetLastError());
  });
}

}  // extern "C"

namespace wc {

// the lattice descriptor and the D work list of one lattice, written into scratch memory
// (kernel arguments instead of a host copy, so that nothing is allocated or staged)
__global__ void k_noalloc_tables(LatDesc L, int nrhs, int nr, LatDesc* lat_out, WorkItem* items) {
  const int nch = L.nchunks;
  const int ngroups = (nrhs + nr - 1) / nr;
  const int n = nch * ngroups;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int grp = i / nch, chunk = i - grp * nch;
    const int r0 = grp * nr;
    items[i] = WorkItem{0, chunk, r0, min(nr, nrhs - r0)};
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *lat_out = L;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace wc

extern "C" {

int wc_apply_D_noalloc(wc_ctx* c, void* out, const void* in, int nrhs, int prec, int region, int dagger,
                       void* stream) {
  return guarded([&] {
    require(c && out && in && nrhs >= 1, WC_ERR_ARG, "null argument or nrhs < 1");
    check_prec(prec);
    require(region == WC_FULL || region == WC_BLOCKS, WC_ERR_ARG, "bad region");
    require(c->have_clover, WC_ERR_STATE, "clover term not created");
    require(c->have_links[prec] && c->have_clov[prec], WC_ERR_STATE,
            "the operator is not resident in this precision: call wc_apply_D once in it first");
    static_assert(sizeof(LatDesc) <= 256, "lattice descriptor exceeds its scratch slot");
    const Geom& g = c->g;
    const int nr = pick_nr(c, nrhs, prec, false, 0);
    const int nch = (g.V + WG - 1) / WG;
    const long long nitems = (long long)nch * ((nrhs + nr - 1) / nr);
    const size_t field = align256(spinor_bytes(prec, (long long)nrhs * g.V));
    const size_t scales = is16(prec) ? align256(sizeof(float) * (size_t)nrhs * g.V) : 0;
    const size_t items_off = 256, in_off = items_off + align256(sizeof(WorkItem) * (size_t)nitems);
    const size_t out_off = in_off + field + scales, need = out_off + field + scales;
    require(need <= SCRATCH_BYTES, WC_ERR_ARG,
            "wc_apply_D_noalloc: " + std::to_string(need >> 20) + " MiB of scratch needed for this lattice, nrhs " +
                "and precision; the limit is " + std::to_string(SCRATCH_BYTES >> 20) + " MiB");
    char* base = (char*)scratch_setup(c->dev);
    hipStream_t st = S(stream);
    LatDesc L;
    std::memset(&L, 0, sizeof L);
    L.g = g;
    L.gauge = c->links[prec].p;
    L.gscale = c->lscale[prec].as<float>();
    L.clov = c->clov[prec].p;
    L.cscale = c->cscale[prec].as<float>();
    L.foff = 0;
    L.nrhs = nrhs;
    L.nchunks = nch;
    L.tiles[0] = c->tiles[0].as<int>();
    L.tiles[1] = c->tiles[1].as<int>();
    L.eo_sites = c->eo_sites.as<short>();
    L.eo_slot = c->eo_slot.as<short>();
    LatDesc* d_lat = (LatDesc*)base;
    WorkItem* d_items = (WorkItem*)(base + items_off);
    hipLaunchKernelGGL(k_noalloc_tables, dim3((unsigned)std::min<long long>((nitems + 255) / 256, 1024)), dim3(256), 0,
                       st, L, nrhs, nr, d_lat, d_items);
    void* fin = base + in_off;
    float* fin_sc = scales ? (float*)(base + in_off + field) : nullptr;
    void* fout = base + out_off;
    float* fout_sc = scales ? (float*)(base + out_off + field) : nullptr;
    launch_pack_spinor(prec, g, nrhs, in, fin, fin_sc, st);
    DiracLaunch a;
    a.lats = d_lat;
    a.items = d_items;
    a.nitems = (int)nitems;
    a.in = fin;
    a.in_sc = fin_sc;
    a.in_prec = prec;
    a.out = fout;
    a.out_sc = fout_sc;
    a.y = nullptr;
    a.y_sc = nullptr;
    a.partials = nullptr;
    a.pw = 0;
    a.skip = nullptr;
    a.dagger = dagger ? 1 : 0;
    a.block = region == WC_BLOCKS;
    // the staging rule of wc_apply_D (a single lattice: its tiles decide)
    const int forced = c->opt_dirac_stage;
    const int stage = g.bvol != 256 ? 0 : (forced >= 0 ? forced : 1);
    a.stage = stage && dirac_stage_lds_bytes(prec, nr) <= LDS_MAX_BYTES;
    launch_dirac(prec, nr, a, persistent_grid(a.nitems, 8), st);
    launch_unpack_spinor(prec, g, nrhs, fout, fout_sc, out, -1, st);
    HIPCK(hipGetLastError());
  });
}

int wc_harmonic_ritz(int m, const void* Hbar, void* theta, void* G) {
  return guarded([&] {
    require(m >= 1 && m <= NKV_MAX && Hbar && theta && G, WC_ERR_ARG, "bad argument");
    require(dense::harmonic_ritz(m, (const dense::cd*)Hbar, m + 1, (dense::cd*)theta, (dense::cd*)G, m),
            WC_ERR_BREAKDOWN, "harmonic Ritz pairs: singular H or no convergence");
  });
}

int wc_sap_block_mr(wc_ctx* c, void* z, void* rho, int nrhs, int colour, int nmr, int prec, int eo, void* stream) {
  return guarded([&] {
    require(c && z && rho && nrhs >= 1 && nmr >= 0, WC_ERR_ARG, "bad argument");
    require(eo == 0 || eo == 1, WC_ERR_ARG, "eo must be 0 or 1");
    require(colour == 0 || colour == 1, WC_ERR_ARG, "colour must be 0 or 1");
    check_prec(prec);
    require(c->have_clover, WC_ERR_STATE, "clover term not created");
    hipStream_t st = S(stream);
    Batch& B = ctx_batch(c, nrhs);
    B.sap_rho.ensure(prec, B.sites_rhs);
    B.sap_z.ensure(prec, B.sites_rhs);
    B.sap_psi.ensure(prec, B.sites_rhs);
    const void* ins[1] = {rho};
    pack_batch(B, prec, ins, B.sap_rho, st);
    run_sap_halfsweep(B, prec, pick_nr(c, nrhs, prec, true, 0, eo), colour, nmr, B.sap_rho, B.sap_z, B.sap_psi, nullptr,
                      1, 0, 1, 1, eo, st);
    void* zo[1] = {z};
    void* ro[1] = {rho};
    unpack_batch(B, prec, B.sap_z, zo, colour, st);
    unpack_batch(B, prec, B.sap_rho, ro, colour, st);
    HIPCK(hipGetLastError());
  });
}

int wc_sap(wc_ctx* c, void* psi, const void* eta, int nrhs, int ncy, int nmr, int prec, int eo, void* stream) {
  return guarded([&] {
    require(c && psi && eta && nrhs >= 1 && ncy >= 1 && nmr >= 0, WC_ERR_ARG, "bad argument");
    require(eo == 0 || eo == 1, WC_ERR_ARG, "eo must be 0 or 1");
    check_prec(prec);
    require(c->have_clover, WC_ERR_STATE, "clover term not created");
    hipStream_t st = S(stream);
    Batch& B = ctx_batch(c, nrhs);
    B.sap_rho.ensure(prec, B.sites_rhs);
    B.sap_z.ensure(prec, B.sites_rhs);
    B.sap_psi.ensure(prec, B.sites_rhs);
    const void* ins[1] = {eta};
    pack_batch(B, prec, ins, B.sap_rho, st);
    run_sap(B, prec, pick_nr(c, nrhs, prec, true, 0, eo), ncy, nmr, B.sap_rho, B.sap_z, B.sap_psi, nullptr, eo, st);
    void* outs[1] = {psi};
    unpack_batch(B, prec, B.sap_psi, outs, -1, st);
    HIPCK(hipGetLastError());
  });
}

// the cached batch of these lattices (argument checks first: a bad list caches nothing)
static Batch* batch_for(const std::vector<wc_ctx*>& cs, const std::vector<int>& ns) {
  for (size_t i = 0; i < cs.size(); ++i) require(cs[i] && ns[i] >= 1, WC_ERR_ARG, "bad lattice argument");
  return cs.size() == 1 ? &ctx_batch(cs[0], ns[0]) : &multi_batch(cs, ns);
}

// kdefl < 0: FGCR; kdefl >= 0: FGMRES-DR keeping kdefl harmonic Ritz vectors
static int solve_batch_impl(const std::vector<wc_ctx*>& ctxs, const std::vector<int>& nrhs, void* const* x,
                            const void* const* b, const wc_solver_params* p, wc_solver_stats* st_out, void* stream,
                            Batch* cached, int kdefl = -1) {
  int rc = WC_OK;
  int grc = guarded([&] {
    require(p, WC_ERR_ARG, "null params");
    int max_nrhs = 0;
    for (size_t i = 0; i < ctxs.size(); ++i) {
      require(ctxs[i] && x[i] && b[i] && nrhs[i] >= 1, WC_ERR_ARG, "bad lattice argument");
      require(ctxs[i]->have_clover, WC_ERR_STATE, "clover term not created");
      max_nrhs = std::max(max_nrhs, nrhs[i]);
    }
    hipStream_t st = S(stream);
    std::unique_ptr<Batch> owned;
    Batch* B = cached;
    if (!B) {
      owned = std::make_unique<Batch>();
      owned->init(ctxs, nrhs);
      B = owned.get();
    }
    SolveSetup s = make_setup(*p, ctxs[0], max_nrhs);
    require(kdefl < s.nkv, WC_ERR_ARG, "FGMRES-DR needs fewer deflated vectors than the cycle length");
    require(kdefl < 0 || (p->basis_prec == WC_F64 && p->drop == 0.0), WC_ERR_ARG,
            "FGMRES-DR keeps an FP64 basis: basis_prec must be WC_F64 and drop 0");
    if (kdefl >= 0)
      prepare_fgmres(*B, s);
    else
      prepare_solver(*B, s);
    pack_batch(*B, P_F64, b, B->b, st);
    if (p->x0_given) pack_batch(*B, P_F64, (const void* const*)x, B->x, st);
    // D^dag x = b  <=>  D (g5 x) = g5 b
    auto gamma5 = [&](Field& f) {
      long long off = 0;
      for (size_t i = 0; i < B->lat.size(); ++i) {
        const long long V = B->lat[i]->g.V;
        launch_gamma5_f64((double2*)f.data() + off * 12, V, B->nrhs[i], st);
        off += (long long)B->nrhs[i] * V;
      }
    };
    if (p->dagger) {
      gamma5(B->b);
      if (p->x0_given) gamma5(B->x);
    }
    std::vector<wc_solver_stats> stats;
    if (kdefl >= 0)
      rc = fgmres_dr_solve(*B, s, kdefl, p->x0_given != 0, p->use_graph != 0, ctxs[0], stats, st);
    else
      rc = fgcr_solve(*B, s, p->x0_given != 0, p->use_graph != 0, ctxs[0], stats, st);
    if (p->dagger) gamma5(B->x);
    unpack_batch(*B, P_F64, B->x, x, -1, st);
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(st));
    if (st_out)
      for (size_t i = 0; i < stats.size(); ++i) st_out[i] = stats[i];
    if (rc != WC_OK) {
      const char* what = kdefl >= 0 ? "FGMRES-DR" : "FGCR";
      bool stagnated = false;
      for (const wc_solver_stats& o : stats) stagnated |= o.stagnated != 0;
      g_last_error = std::string(what) + (rc == WC_ERR_BREAKDOWN ? " breakdown"
                                          : stagnated ? " stagnated: the true residual did not drop over "
                                                            + std::to_string(p->stag) + " restarts"
                                                      : " did not converge within maxit");
    }
  });
  return grc != WC_OK ? grc : rc;
}

int wc_fgcr_solve(wc_ctx* c, void* x, const void* b, int nrhs, const wc_solver_params* p, wc_solver_stats* st,
                  void* stream) {
  if (!c || nrhs < 1) {
    g_last_error = "null context or nrhs < 1";
    return WC_ERR_ARG;
  }
  Batch* B = nullptr;
  int rc = guarded([&] { B = &ctx_batch(c, nrhs); });
  if (rc != WC_OK) return rc;
  void* xs[1] = {x};
  const void* bs[1] = {b};
  return solve_batch_impl({c}, {nrhs}, xs, bs, p, st, stream, B);
}

int wc_fgmres_dr_solve(wc_ctx* c, void* x, const void* b, int nrhs, const wc_solver_params* p, int kdefl,
                       wc_solver_stats* st, void* stream) {
  if (!c || nrhs < 1 || kdefl < 0) {
    g_last_error = "null context, nrhs < 1 or kdefl < 0";
    return WC_ERR_ARG;
  }
  Batch* B = nullptr;
  int rc = guarded([&] { B = &ctx_batch(c, nrhs); });
  if (rc != WC_OK) return rc;
  void* xs[1] = {x};
  const void* bs[1] = {b};
  return solve_batch_impl({c}, {nrhs}, xs, bs, p, st, stream, B, kdefl);
}

int wc_fgcr_solve_batch(wc_ctx* const* ctxs, int nlat, void* const* x, const void* const* b, const int* nrhs,
                        const wc_solver_params* p, wc_solver_stats* st, void* stream) {
  if (!ctxs || nlat < 1 || !x || !b || !nrhs) {
    g_last_error = "null argument";
    return WC_ERR_ARG;
  }
  std::vector<wc_ctx*> cs(ctxs, ctxs + nlat);
  std::vector<int> ns(nrhs, nrhs + nlat);
  Batch* B = nullptr;
  int rc = guarded([&] { B = batch_for(cs, ns); });
  if (rc != WC_OK) return rc;
  return solve_batch_impl(cs, ns, x, b, p, st, stream, B);
}

int wc_fgmres_dr_solve_batch(wc_ctx* const* ctxs, int nlat, void* const* x, const void* const* b, const int* nrhs,
                             const wc_solver_params* p, int kdefl, wc_solver_stats* st, void* stream) {
  if (!ctxs || nlat < 1 || !x || !b || !nrhs || kdefl < 0) {
    g_last_error = "null argument or kdefl < 0";
    return WC_ERR_ARG;
  }
  std::vector<wc_ctx*> cs(ctxs, ctxs + nlat);
  std::vector<int> ns(nrhs, nrhs + nlat);
  Batch* B = nullptr;
  int rc = guarded([&] { B = batch_for(cs, ns); });
  if (rc != WC_OK) return rc;
  return solve_batch_impl(cs, ns, x, b, p, st, stream, B, kdefl);
}

int wc_link_grad(wc_ctx* c, void* G, const void* Y, const void* X, int nrhs, double coef, void* stream) {
  return guarded([&] {
    require(c && G && Y && X && nrhs >= 1, WC_ERR_ARG, "bad argument");
    DevBuf xi;
    if (c->csw != 0.0) xi.ensure(sizeof(double2) * 54 * (size_t)c->g.V);
    launch_force(c->dims, c->bc_t, c->Ucanon.p, Y, X, nrhs, c->have_clover ? c->csw : 0.0, coef, 0, xi.p, G,
                 S(stream));
    HIPCK(hipGetLastError());
    HIPCK(hipStreamSynchronize(S(stream)));
  });
}

// Y = D^-dag phi = g5 D^-1 g5 phi (gamma5-hermiticity), then X = D^-1 Y, into the
// caller's or the library's buffers; returns the first solve status that is not WC_OK.
static int action_solves(wc_ctx* c, const void* phi, const wc_solver_params* p, void* y, void* x, void* tmp,
                         wc_solver_stats* s2, void* stream) {
  hipStream_t st_ = S(stream);
  wc_solver_params q = *p;
  q.x0_given = 0;
  q.dagger = 0;
  launch_gamma5_canon(c->g.V, phi, tmp, st_);
  const int r1 = wc_fgcr_solve(c, y, tmp, 1, &q, &s2[0], stream);
  require(r1 == WC_OK || r1 == WC_ERR_NOT_CONVERGED || r1 == WC_ERR_BREAKDOWN, r1, g_last_error);
  launch_gamma5_canon(c->g.V, y, y, st_);
  const int r2 = wc_fgcr_solve(c, x, y, 1, &q, &s2[1], stream);
  require(r2 == WC_OK || r2 == WC_ERR_NOT_CONVERGED || r2 == WC_ERR_BREAKDOWN, r2, g_last_error);
  return r1 != WC_OK ? r1 : r2;
}

int wc_force(wc_ctx* c, void* F, const void* phi, const wc_solver_params* p, wc_solver_stats* st, void* Yout,
             void* Xout, void* stream) {
  int rc_solve = WC_OK;
  int rc = guarded([&] {
    require(c && F && phi && p, WC_ERR_ARG, "bad argument");
    require(c->have_clover, WC_ERR_STATE, "clover term not created");
    hipStream_t st_ = S(stream);
    const size_t bytes = (size_t)c->g.V * 192;
    DevBuf y, x, tmp;
    y.ensure(bytes);
    x.ensure(bytes);
    tmp.ensure(bytes);
    wc_solver_stats s2[2];
    rc_solve = action_solves(c, phi, p, y.p, x.p, tmp.p, s2, stream);
    DevBuf xi;
    if (c->csw != 0.0) xi.ensure(sizeof(double2) * 54 * (size_t)c->g.V);
    launch_force(c->dims, c->bc_t, c->Ucanon.p, y.p, x.p, 1, c->csw, 1.0, 1, xi.p, F, st_);
    HIPCK(hipGetLastError());
    if (Yout) HIPCK(hipMemcpyAsync(Yout, y.p, bytes, hipMemcpyDeviceToDevice, st_));
    if (Xout) HIPCK(hipMemcpyAsync(Xout, x.p, bytes, hipMemcpyDeviceToDevice, st_));
    HIPCK(hipStreamSynchronize(st_));
    if (st) {
      st[0] = s2[0];
      st[1] = s2[1];
    }
  });
  return rc != WC_OK ? rc : rc_solve;
}

int wc_pseudofermion_action(wc_ctx* c, const void* phi, const wc_solver_params* p, double* Sout, void* Y, void* X,
                            wc_solver_stats* st, void* stream) {
  int rc_solve = WC_OK;
  int rc = guarded([&] {
    require(c && phi && p && Sout && Y && X, WC_ERR_ARG, "bad argument");
    require(c->have_clover, WC_ERR_STATE, "clover term not created");
    hipStream_t st_ = S(stream);
    DevBuf tmp, work;
    tmp.ensure((size_t)c->g.V * 192);
    work.ensure(sizeof(double) * 1025);
    wc_solver_stats s2[2];
    rc_solve = action_solves(c, phi, p, Y, X, tmp.p, s2, stream);
    launch_norm2_canon((long long)c->g.V * 12, Y, work.as<double>(), st_);
    HIPCK(hipGetLastError());
    HIPCK(hipMemcpyAsync(Sout, work.p, sizeof(double), hipMemcpyDeviceToHost, st_));
    HIPCK(hipStreamSynchronize(st_));
    if (st) {
      st[0] = s2[0];
      st[1] = s2[1];
    }
  });
  return rc != WC_OK ? rc : rc_solve;
}

int wc_spinor_scale(wc_ctx* c, void* out, const void* in, int nrhs, double coef, void* stream) {
  return guarded([&] {
    require(c && out && in && nrhs >= 1, WC_ERR_ARG, "bad argument");
    launch_scale_canon((long long)c->g.V * 12 * nrhs, coef, in, out, S(stream));
    HIPCK(hipGetLastError());
  });
}

// Mean time per launch of f: `iters` launches captured into one hipGraph (so host-side
// launch overhead does not enter), replayed between two events on `st`.
static double time_launches(wc_ctx* c, hipStream_t st, int iters, const std::function<void(hipStream_t)>& f) {
  f(st);  // warm-up (twice: alternating launches such as the two SAP colours) creates
  f(st);  // every buffer and work list the captured launches touch
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(st));
  if (!c->cap) HIPCK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  struct Exec {
    hipGraphExec_t g;
    ~Exec() { (void)hipGraphExecDestroy(g); }
  } exec{capture_graph(c->cap, [&](hipStream_t cs) {
    for (int i = 0; i < iters; ++i) f(cs);
  })};
  HipEvent e0, e1;
  HIPCK(hipGraphLaunch(exec.g, st));
  HIPCK(hipEventRecord(e0, st));
  HIPCK(hipGraphLaunch(exec.g, st));
  HIPCK(hipEventRecord(e1, st));
  HIPCK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCK(hipEventElapsedTime(&ms, e0, e1));
  return double(ms) / iters;
}

int wc_bench_dirac(wc_ctx* c, int prec, int nrhs, int region, int iters, double* ms, void* stream) {
  return guarded([&] {
    require(c && ms && nrhs >= 1 && iters >= 1, WC_ERR_ARG, "bad argument");
    check_prec(prec);
    require(c->have_clover, WC_ERR_STATE, "clover term not created");
    hipStream_t st = S(stream);
    Batch& B = ctx_batch(c, nrhs);
    B.ain[prec].ensure(prec, B.sites_rhs);
    B.aout[prec].ensure(prec, B.sites_rhs);
    HIPCK(hipMemsetAsync(B.ain[prec].data(), 0, spinor_bytes(prec, B.sites_rhs), st));
    if (B.ain[prec].scale()) HIPCK(hipMemsetAsync(B.ain[prec].scale(), 0, sizeof(float) * B.sites_rhs, st));
    const int nr = pick_nr(c, nrhs, prec, false, 0);
    *ms = time_launches(c, st, iters, [&](hipStream_t s) {
      run_dirac(B, prec, nr, B.ain[prec], B.aout[prec], nullptr, nullptr, nullptr, 0, region == WC_BLOCKS, s);
    });
    HIPCK(hipGetLastError());
  });
}

int wc_bench_sap(wc_ctx* c, int prec, int nrhs, int nmr, int eo, int iters, double* ms, void* stream) {
  return guarded([&] {
    require(c && ms && nrhs >= 1 && iters >= 1 && nmr >= 0, WC_ERR_ARG, "bad argument");
    require(eo == 0 || eo == 1, WC_ERR_ARG, "eo must be 0 or 1");
    check_prec(prec);
    require(c->have_clover, WC_ERR_STATE, "clover term not created");
    hipStream_t st = S(stream);
    Batch& B = ctx_batch(c, nrhs);
    B.sap_rho.ensure(prec, B.sites_rhs);
    B.sap_z.ensure(prec, B.sites_rhs);
    B.sap_psi.ensure(prec, B.sites_rhs);
    HIPCK(hipMemsetAsync(B.sap_rho.data(), 0, spinor_bytes(prec, B.sites_rhs), st));
    HIPCK(hipMemsetAsync(B.sap_z.data(), 0, spinor_bytes(prec, B.sites_rhs), st));
    if (B.sap_rho.scale()) {
      HIPCK(hipMemsetAsync(B.sap_rho.scale(), 0, sizeof(float) * B.sites_rhs, st));
      HIPCK(hipMemsetAsync(B.sap_z.scale(), 0, sizeof(float) * B.sites_rhs, st));
    }
    const int nr = pick_nr(c, nrhs, prec, true, 0, eo);
    B.lats(prec, st, eo != 0);
    HIPCK(hipStreamSynchronize(st));
    int colour = 0;
    *ms = time_launches(c, st, iters, [&](hipStream_t s) {
      // a half-sweep as the solver's later cycles run it (border update, odd residual implicit)
      run_sap_halfsweep(B, prec, nr, colour, nmr, B.sap_rho, B.sap_z, B.sap_psi, nullptr, 0, 1, 1, 1, eo, s, 2);
      colour ^= 1;
    });
    HIPCK(hipGetLastError());
  });
}

int wc_autotune(wc_ctx* c, int nrhs, int prec, int nr_out[4], void* stream) {
  return guarded([&] {
    require(c && nrhs >= 1, WC_ERR_ARG, "bad argument");
    check_prec(prec);
    const int cands[4] = {1, 2, 3, 4};
    // D tiles: in prec and, for the outer solver, in FP64 and (16-bit prec) in FP32, the D
    // of the recursion over an F32 basis
    std::vector<int> dps = {prec};
    if (prec != P_F64) dps.push_back(P_F64);
    if (is16(prec)) dps.push_back(P_F32);
    for (int dp : dps) {
      double best = 1e30;
      int nd = 1;
      for (int nr : cands) {
        if (nr > nrhs) continue;
        c->nr_dirac[dp] = nr;
        double t = 0;
        const int rc = wc_bench_dirac(c, dp, nrhs, WC_FULL, 20, &t, stream);
        require(rc == WC_OK, rc, g_last_error);
        if (t < best) {
          best = t;
          nd = nr;
        }
      }
      c->nr_dirac[dp] = nd;
    }
    // block-solver tiles of both block solvers in prec
    double best_s = 1e30, best_e = 1e30;
    int ns = 1, ne = 1;
    for (int nr : cands) {
      if (nr > nrhs || nr > (prec == P_F64 ? 1 : 2)) continue;
      double t = 0;
      c->nr_sap[prec] = nr;
      int rc = wc_bench_sap(c, prec, nrhs, 4, 0, 10, &t, stream);
      require(rc == WC_OK, rc, g_last_error);
      if (t < best_s) {
        best_s = t;
        ns = nr;
      }
      c->nr_sap_eo[prec] = nr;
      rc = wc_bench_sap(c, prec, nrhs, 4, 1, 10, &t, stream);
      require(rc == WC_OK, rc, g_last_error);
      if (t < best_e) {
        best_e = t;
        ne = nr;
      }
    }
    c->nr_sap[prec] = ns;
    c->nr_sap_eo[prec] = ne;
    if (nr_out) {
      nr_out[0] = c->nr_dirac[prec];
      nr_out[1] = c->nr_dirac[P_F64];
      nr_out[2] = ns;
      nr_out[3] = ne;
    }
  });
}

int wc_autotune_block(wc_ctx* c, const wc_solver_params* p, int block_out[4], void* stream) {
  return guarded([&] {
    require(c && p, WC_ERR_ARG, "bad argument");
    require(c->have_clover, WC_ERR_STATE, "clover term not created");
    hipStream_t st = S(stream);
    // candidate shapes: every axis a divisor b of L with an even block count, b <= 8,
    // 16 <= volume <= 256
    std::vector<std::array<int, 4>> cands;
    std::vector<int> divs[4];
    for (int m = 0; m < 4; ++m)
      for (int b = 1; b <= 8; ++b)
        if (c->dims[m] % b == 0 && (c->dims[m] / b) % 2 == 0) divs[m].push_back(b);
    for (int b0 : divs[0])
      for (int b1 : divs[1])
        for (int b2 : divs[2])
          for (int b3 : divs[3]) {
            const int vol = b0 * b1 * b2 * b3;
            // keep near-isotropic shapes (spatial extents equal, time extent within 2x)
            if (vol < 16 || vol > 256 || b1 != b2 || b2 != b3 || b0 > 2 * b1 || b1 > 2 * b0) continue;
            cands.push_back({b0, b1, b2, b3});
          }
    require(!cands.empty(), WC_ERR_GEOMETRY, "no valid block shape for this lattice");
    const size_t bytes = (size_t)c->g.V * 192;
    DevBuf bsrc, xsol;
    bsrc.ensure(bytes);
    xsol.ensure(bytes);
    launch_fill_hash((long long)c->g.V * 12, 12345u, bsrc.p, st);
    HIPCK(hipGetLastError());
    double best = 1e300;
    std::array<int, 4> best_b = {c->block[0], c->block[1], c->block[2], c->block[3]};
    for (auto& b : cands) {
      layout(c, b.data(), st);
      wc_solver_params q = *p;
      q.x0_given = 0;
      q.dagger = 0;
      wc_solver_stats sst;
      // first solve builds graphs and buffers; the second is timed
      int rc = wc_fgcr_solve(c, xsol.p, bsrc.p, 1, &q, &sst, stream);
      if (rc != WC_OK && rc != WC_ERR_NOT_CONVERGED) continue;
      rc = wc_fgcr_solve(c, xsol.p, bsrc.p, 1, &q, &sst, stream);
      if (rc != WC_OK) continue;
      if (sst.time_ms < best) {
        best = sst.time_ms;
        best_b = b;
      }
    }
    layout(c, best_b.data(), st);
    if (block_out)
      for (int m = 0; m < 4; ++m) block_out[m] = best_b[m];
  });
}

const char* wc_last_error(void) { return g_last_error.c_str(); }

int wc_version(void) { return 201; }

void wc_destroy(wc_ctx* c) { delete c; }

}  // extern "C"
