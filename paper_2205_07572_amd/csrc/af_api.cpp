// af_api.cpp -- C ABI of libaf.so (declared in include/af.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "af.h"
#include "af_hier.h"
#include "af_internal.h"
#include "af_launch.h"
#include "af_probe.h"
#include "af_weights.h"

using namespace af;

namespace {

thread_local std::string g_err;

af_status fail(af_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define AF_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) return fail(AF_ERR_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

// Device memory for the tables of a context's hierarchies.  A regrid builds
// a new hierarchy of about the size of the old one every few coarse steps;
// its tables reuse the old one's blocks instead of a hipMalloc per table and
// a hipFree per table, which drains the device.  Blocks come in power-of-two
// capacities.  Shared by the context and its hierarchies and freed with the
// last of them.
struct DevPool {
  std::multimap<size_t, void*> idle;  // capacity -> block not in use
  std::map<void*, size_t> cap;        // every block -> capacity
  ~DevPool() {
    for (auto& b : cap) (void)hipFree(b.first);
  }
  hipError_t get(void** p, size_t bytes) {
    size_t c = 256;
    while (c < bytes) c <<= 1;
    auto it = idle.find(c);
    if (it != idle.end()) {
      *p = it->second;
      idle.erase(it);
      return hipSuccess;
    }
    const hipError_t e = hipMalloc(p, c);
    if (e == hipSuccess) cap[*p] = c;
    return e;
  }
  // back to the pool; the caller has made sure no queued work reads it
  void put(void* p) {
    auto it = p ? cap.find(p) : cap.end();
    if (it != cap.end()) idle.emplace(it->second, p);
  }
};

struct af_ctx {
  af_problem P;
  std::shared_ptr<DevPool> pool = std::make_shared<DevPool>();
  int ncomp;
  int ty = 0;  // step tile height (rows per block)
  bool fused_pairs = true;  // batched coarse step: fused pairs of finest-level substeps
  int adv_k = 0, adv_nt = 0;  // level-advance steps per launch and block size (0 = default)
  // fill-set entries of one patch block (device); the first ninner lie
  // within one cell of the interior (all an interior-region step reads)
  std::vector<int32_t> h_entries;
  int32_t* d_entries = nullptr;  // uploaded on first device use
  int nentries = 0, ninner = 0;
  // indices of the entries that are nodes on the closed square [0, m]^2
  std::vector<int32_t> h_bnd;
  int32_t* d_bnd = nullptr;
  // coarse -> fine fill weights (device)
  FillWeights* d_fillw = nullptr;
  // reduction workspace
  double* d_part = nullptr;
  int part_cap = 0;
  // weights cache keyed by (dt/dx, dt/dy)
  std::map<std::pair<double, double>, std::vector<unsigned char>> wcache;
  // device copies of the acoustic orbit weights (the batched step reads them
  // through a pointer), keyed like wcache
  std::map<std::pair<double, double>, void*> wdev;

  double dx(int l) const { return P.lx / double(P.n0x * P.m) / double(1 << l); }
  double dy(int l) const { return P.ly / double(P.n0y * P.m) / double(1 << l); }
  bool fp32() const { return P.prec == AF_FP32; }
  size_t elem() const { return fp32() ? 4 : 8; }
};

constexpr size_t kMaxGraphs = 64;  // executable graphs kept per hierarchy

struct GraphKey {
  uint32_t mask;
  double dt0;
  const void* b0;
  const void* b1;
  const double* reg;
  double t0;    // only for time-dependent fields (else 0)
  int32_t flags;
  bool operator<(const GraphKey& o) const {
    return std::tie(mask, dt0, b0, b1, reg, t0, flags) < std::tie(o.mask, o.dt0, o.b0, o.b1, o.reg, o.t0, o.flags);
  }
};

struct af_hier {
  af_ctx* ctx = nullptr;
  std::shared_ptr<DevPool> pool;  // the context's (the tables below come from it)
  Hier H;
  int32_t* d_lut = nullptr;
  int32_t* d_level = nullptr;
  int32_t* d_ix = nullptr;
  int32_t* d_iy = nullptr;
  uint8_t* d_side_mask = nullptr;
  int32_t* d_xy = nullptr;     // [n][2] (ix, iy)
  CFFace* d_faces = nullptr;
  std::vector<int> face_off;  // per coarse level offset into d_faces
  std::vector<CFFace> all_faces;
  bool on_device = false;     // tables are uploaded on first device use
  // per level: -1 not checked, 1 the level is the complete row-major patch
  // array (the level advance can run on it), 0 otherwise
  std::vector<int> nbr_ok;
  HierDev dev{};
  std::map<GraphKey, hipGraphExec_t> graphs;
  // ghost-fill plans per lowest source level (built on first use)
  std::vector<int4*> d_plan;
  std::vector<uint32_t*> d_plan_flags;
  std::vector<int4*> d_canon_ops;  // per source bound: the vertex copies of k_amr_sync
  // with the plan of source bound 0: same-level neighbours [n][9] and the
  // directions the batched step stages by a same-level gather [n]
  int32_t* d_nbr = nullptr;
  uint32_t* d_gnflags = nullptr;
  // leaves with a neighbour of another level (the only ones a coarser
  // reconstruction can read from), in leaf order; those of level >= l are
  // impure[impure_off[l] ..]
  std::vector<int32_t> impure;
  std::vector<int> impure_off;
  int32_t* d_impure = nullptr;
};

namespace {

template <typename T>
T* dev_upload(const std::vector<T>& v, hipError_t* err) {
  T* p = nullptr;
  const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
  *err = hipMalloc(&p, bytes);
  if (*err != hipSuccess) return nullptr;
  if (!v.empty()) *err = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return p;
}

// dev_upload into a block of the pool
template <typename T>
T* pool_upload(DevPool& pool, const std::vector<T>& v, hipError_t* err) {
  void* p = nullptr;
  *err = pool.get(&p, std::max<size_t>(1, v.size()) * sizeof(T));
  if (*err != hipSuccess) return nullptr;
  if (!v.empty()) *err = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return static_cast<T*>(p);
}

af_status check_state(const af_ctx* c, const af_state* s, int need_patches, const char* what) {
  if (!s) return fail(AF_ERR_ARG, std::string(what) + ": null state");
  for (int k = 0; k < 4; ++k)
    if (!s->dof[k]) return fail(AF_ERR_ARG, std::string(what) + ": null DOF array");
  if (s->pitch < c->P.m + 5) return fail(AF_ERR_LAYOUT, std::string(what) + ": pitch < m+5");
  if (s->npatch < need_patches) return fail(AF_ERR_LAYOUT, std::string(what) + ": state holds too few patches");
  for (int k = 0; k < 4; ++k)
    if (reinterpret_cast<uintptr_t>(s->dof[k]) % c->elem() != 0)
      return fail(AF_ERR_LAYOUT, std::string(what) + ": misaligned DOF array");
  return AF_OK;
}

af_status check_cfl(const af_ctx* c, int level, double dt) {
  if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(AF_ERR_ARG, "dt must be finite and >= 0");
  const double dx = c->dx(level), dy = c->dy(level);
  if (c->P.eq == AF_ADVECTION) {
    const double cfl = std::max(std::fabs(c->P.a) * dt / dx, std::fabs(c->P.b) * dt / dy);
    if (cfl > 1.0 + 1e-12) return fail(AF_ERR_CFL, "advection CFL > 1 (eq. cfl-adv)");
  } else if (c->P.eq == AF_SWIRL) {
    // |a|, |b| <= max |grad Psi| = 1 (centred differences of Psi keep the bound)
    const double cfl = std::max(dt / dx, dt / dy);
    if (cfl > 1.0 + 1e-12) return fail(AF_ERR_CFL, "swirl CFL > 1 (eq. cfl-adv with |a|, |b| <= 1)");
  } else if (c->P.eq == AF_BURGERS) {
    // the speed is q in both directions, |q| <= qmax
    const double cfl = c->P.qmax * std::max(dt / dx, dt / dy);
    if (cfl > 1.0 + 1e-12) return fail(AF_ERR_CFL, "Burgers CFL > 1 (qmax dt / dx)");
  } else if (c->P.eq == AF_ROTATION) {
    // largest |a| = |omega| |y - yc| and |b| = |omega| |x - xc| on the domain
    const double w = std::fabs(c->P.omega);
    const double amax = w * std::max(std::fabs(c->P.y0 - c->P.yc), std::fabs(c->P.y0 + c->P.ly - c->P.yc));
    const double bmax = w * std::max(std::fabs(c->P.x0 - c->P.xc), std::fabs(c->P.x0 + c->P.lx - c->P.xc));
    const double cfl = std::max(amax * dt / dx, bmax * dt / dy);
    if (cfl > 1.0 + 1e-12) return fail(AF_ERR_CFL, "rotation CFL > 1 (eq. cfl-adv with the largest speed)");
  } else {
    const double cfl = c->P.c * dt / std::min(dx, dy);
    if (cfl > 0.5 + 1e-12) return fail(AF_ERR_CFL, "acoustic CFL > 1/2 (eq. cfl-acoustics)");
  }
  return AF_OK;
}

const void* weights_for(af_ctx* c, double dtdx, double dtdy) {
  auto key = std::make_pair(dtdx, dtdy);
  auto it = c->wcache.find(key);
  if (it != c->wcache.end()) return it->second.data();
  std::vector<unsigned char> buf;
  if (c->P.eq == AF_ADVECTION) {
    if (c->fp32()) {
      buf.resize(sizeof(AdvWeights<float>));
      make_adv_weights<float>(c->P.a * dtdx, c->P.b * dtdy, reinterpret_cast<AdvWeights<float>*>(buf.data()));
    } else {
      buf.resize(sizeof(AdvWeights<double>));
      make_adv_weights<double>(c->P.a * dtdx, c->P.b * dtdy, reinterpret_cast<AdvWeights<double>*>(buf.data()));
    }
  } else {
    bool sym;
    if (c->fp32()) {
      buf.resize(sizeof(AcAllWeights<float>));
      auto* W = reinterpret_cast<AcAllWeights<float>*>(buf.data());
      make_ac_weights<float>(c->P.c * dtdx, c->P.c * dtdy, &W->dense);
      sym = make_ac_orbit_weights<float>(c->P.c * dtdx, c->P.c * dtdy, &W->orbit);
    } else {
      buf.resize(sizeof(AcAllWeights<double>));
      auto* W = reinterpret_cast<AcAllWeights<double>*>(buf.data());
      make_ac_weights<double>(c->P.c * dtdx, c->P.c * dtdy, &W->dense);
      sym = make_ac_orbit_weights<double>(c->P.c * dtdx, c->P.c * dtdy, &W->orbit);
    }
    if (!sym) return nullptr;  // cannot happen: the sector means are mirror symmetric
  }
  auto res = c->wcache.emplace(key, std::move(buf));
  return res.first->second.data();
}

// The acoustic orbit weights of weights_for on the device (made on first use
// of a key, outside any graph capture); null on a device error.
const void* weights_dev_for(af_ctx* c, double dtdx, double dtdy) {
  auto key = std::make_pair(dtdx, dtdy);
  auto it = c->wdev.find(key);
  if (it != c->wdev.end()) return it->second;
  const void* host = weights_for(c, dtdx, dtdy);
  if (!host || c->P.eq != AF_ACOUSTICS) return nullptr;
  const void* src = c->fp32() ? static_cast<const void*>(&static_cast<const AcAllWeights<float>*>(host)->orbit)
                              : static_cast<const void*>(&static_cast<const AcAllWeights<double>*>(host)->orbit);
  const size_t bytes = c->fp32() ? sizeof(AcOrbitWeights<float>) : sizeof(AcOrbitWeights<double>);
  void* d = nullptr;
  if (hipMalloc(&d, bytes) != hipSuccess) return nullptr;
  if (hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return nullptr;
  }
  c->wdev.emplace(key, d);
  return d;
}

BufLaunch make_buf(const af_ctx* c, const af_state* b0, const af_state* b1, uint32_t mask) {
  BufLaunch B;
  for (int k = 0; k < 4; ++k) {
    B.p[0][k] = b0->dof[k];
    B.p[1][k] = b1->dof[k];
  }
  B.npatch = b0->npatch;
  B.pitch = b0->pitch;
  B.m = c->P.m;
  B.ncomp = c->ncomp;
  B.mask = mask;
  return B;
}

af_status ctx_device(af_ctx* c) {
  if (c->d_entries) return AF_OK;
  hipError_t err;
  std::vector<FillWeights> fw(1);
  make_fill_weights(&fw[0]);
  c->d_fillw = dev_upload(fw, &err);
  if (err == hipSuccess) c->d_entries = dev_upload(c->h_entries, &err);
  if (err == hipSuccess) c->d_bnd = dev_upload(c->h_bnd, &err);
  if (err != hipSuccess) return fail(AF_ERR_DEVICE, std::string("fill table upload: ") + hipGetErrorString(err));
  return AF_OK;
}

af_status hier_device(af_hier* h) {
  if (h->on_device) return AF_OK;
  const int n = int(h->H.leaves.size());
  std::vector<int32_t> lv(n), vx(n), vy(n), xy(2 * size_t(n));
  for (int k = 0; k < n; ++k) {
    lv[k] = h->H.leaves[k].level;
    vx[k] = h->H.leaves[k].ix;
    vy[k] = h->H.leaves[k].iy;
    xy[2 * k] = vx[k];
    xy[2 * k + 1] = vy[k];
  }
  hipError_t err;
  DevPool& pool = *h->pool;
  h->d_lut = pool_upload(pool, h->H.lut, &err);
  if (err == hipSuccess) h->d_level = pool_upload(pool, lv, &err);
  if (err == hipSuccess) h->d_ix = pool_upload(pool, vx, &err);
  if (err == hipSuccess) h->d_iy = pool_upload(pool, vy, &err);
  if (err == hipSuccess) h->d_side_mask = pool_upload(pool, h->H.side_mask, &err);
  if (err == hipSuccess) h->d_xy = pool_upload(pool, xy, &err);
  if (err == hipSuccess) h->d_faces = pool_upload(pool, h->all_faces, &err);
  if (err == hipSuccess) h->d_impure = pool_upload(pool, h->impure, &err);
  if (err != hipSuccess) return fail(AF_ERR_DEVICE, std::string("hierarchy upload: ") + hipGetErrorString(err));
  HierDev& D = h->dev;
  D.lut = h->d_lut;
  D.plevel = h->d_level;
  D.pix = h->d_ix;
  D.piy = h->d_iy;
  for (int l = 0; l < kMaxLevels; ++l) D.lut_off[l] = (l <= h->H.lmax) ? h->H.lut_off[l] : 0;
  D.npx0 = h->H.n0x;
  D.npy0 = h->H.n0y;
  D.lmax = h->H.lmax;
  D.nleaves = n;
  h->on_device = true;
  return AF_OK;
}

af_status check_pair(const af_ctx* c, const af_hier* h, const af_state* bufs, const char* what) {
  if (!bufs) return fail(AF_ERR_ARG, std::string(what) + ": null buffers");
  const int n = int(h->H.leaves.size());
  af_status s = check_state(c, &bufs[0], n, what);
  if (s != AF_OK) return s;
  s = check_state(c, &bufs[1], n, what);
  if (s != AF_OK) return s;
  if (bufs[0].npatch != bufs[1].npatch || bufs[0].pitch != bufs[1].pitch)
    return fail(AF_ERR_LAYOUT, std::string(what) + ": the two buffers differ in layout");
  return AF_OK;
}

}  // namespace

extern "C" {

const char* af_last_error(void) { return g_err.c_str(); }

af_status af_ctx_create(const af_problem* prob, af_ctx** out) {
  if (!prob || !out) return fail(AF_ERR_ARG, "null argument");
  const af_problem& P = *prob;
  if (P.eq != AF_ADVECTION && P.eq != AF_ACOUSTICS && P.eq != AF_ROTATION && P.eq != AF_SWIRL &&
      P.eq != AF_BURGERS)
    return fail(AF_ERR_ARG, "unknown equation");
  if (P.eq == AF_ROTATION && !(std::isfinite(P.omega) && std::isfinite(P.xc) && std::isfinite(P.yc)))
    return fail(AF_ERR_ARG, "rotation parameters must be finite");
  if (P.prec != AF_FP64 && P.prec != AF_FP32) return fail(AF_ERR_ARG, "unknown precision");
  if (!(P.m == 8 || P.m == 16 || P.m == 32 || P.m == 64 || P.m == 128))
    return fail(AF_ERR_ARG, "m must be 8, 16, 32, 64 or 128");
  if (P.n0x < 1 || P.n0y < 1 || P.lmax < 0 || P.lmax >= kMaxLevels) return fail(AF_ERR_ARG, "bad patch counts or lmax");
  if (!(P.lx > 0 && P.ly > 0)) return fail(AF_ERR_ARG, "domain extents must be positive");
  if (P.eq == AF_ACOUSTICS && !(P.c > 0)) return fail(AF_ERR_ARG, "speed of sound must be positive");
  if (P.eq == AF_BURGERS && !(P.qmax > 0 && std::isfinite(P.qmax)))
    return fail(AF_ERR_ARG, "AF_BURGERS needs a finite bound qmax > 0 on |q| (CFL check)");
  auto c = std::make_unique<af_ctx>();
  c->P = P;
  c->ncomp = P.eq == AF_ACOUSTICS ? 3 : 1;
  // default tile heights: about 256 cells per block, smaller for FP64
  // acoustics at m >= 32 (LDS); a whole 16^2 patch per block is the faster
  // shape in both precisions
  const bool big = (P.eq == AF_ACOUSTICS && P.prec == AF_FP64);
  switch (P.m) {
    case 8: c->ty = 8; break;
    case 16: c->ty = 16; break;
    case 32: c->ty = big ? 4 : 8; break;
    case 64: c->ty = big ? 2 : 4; break;
    default: c->ty = 2; break;
  }
  // fill-set entries: every block DOF except interior averages and nodes
  // strictly inside the interior square.  Those within one cell of the
  // interior (cells [-1, m], nodes [-1, m+1]: what a step of the interior
  // region reads) come first.
  std::vector<int32_t> ent;
  const int m = P.m;
  for (int ring = 0; ring < 2; ++ring)
    for (int kind = 0; kind < 4; ++kind) {
      const int ihi = (kind == 0 || kind == 3) ? m + 1 : m + 2;
      const int jhi = (kind == 0 || kind == 2) ? m + 1 : m + 2;
      for (int j = -2; j <= jhi; ++j)
        for (int i = -2; i <= ihi; ++i) {
          bool inside;
          if (kind == 0) inside = i >= 0 && i < m && j >= 0 && j < m;
          else if (kind == 1) inside = i >= 1 && i <= m - 1 && j >= 1 && j <= m - 1;
          else if (kind == 2) inside = i >= 1 && i <= m - 1 && j >= 0 && j <= m - 1;
          else inside = i >= 0 && i <= m - 1 && j >= 1 && j <= m - 1;
          if (inside) continue;
          const bool inner = i >= -1 && i <= ihi - 1 && j >= -1 && j <= jhi - 1;
          if (inner != (ring == 0)) continue;
          const bool closed = kind > 0 && i >= 0 && i <= ihi - 2 && j >= 0 && j <= jhi - 2;
          if (closed) c->h_bnd.push_back(int32_t(ent.size()));
          ent.push_back((kind << 24) | ((i + 2) << 12) | (j + 2));
        }
      if (ring == 0 && kind == 3) c->ninner = int(ent.size());
    }
  c->h_entries = std::move(ent);
  c->nentries = int(c->h_entries.size());
  *out = c.release();
  return AF_OK;
}

af_status af_ctx_destroy(af_ctx* ctx) {
  if (!ctx) return AF_OK;
  (void)hipFree(ctx->d_entries);
  (void)hipFree(ctx->d_bnd);
  (void)hipFree(ctx->d_fillw);
  (void)hipFree(ctx->d_part);
  for (auto& w : ctx->wdev) (void)hipFree(w.second);
  delete ctx;
  return AF_OK;
}

af_status af_fma_probe(int32_t prec, void* out, int32_t nblocks, int32_t iters, hipStream_t stream) {
  if (prec != AF_FP32 && prec != AF_FP64) return fail(AF_ERR_ARG, "af_fma_probe: precision must be AF_FP32 or AF_FP64");
  if (!out || nblocks < 1 || iters < 1) return fail(AF_ERR_ARG, "af_fma_probe: need out, nblocks >= 1, iters >= 1");
  AF_HIP(launch_fma_probe(prec == AF_FP32, out, nblocks, iters, stream));
  return AF_OK;
}

af_status af_ctx_set_tile(af_ctx* ctx, int32_t ty) {
  if (!ctx) return fail(AF_ERR_ARG, "null ctx");
  if (!step_shape_supported(ctx->P.m, ty)) return fail(AF_ERR_ARG, "unsupported tile height for this m");
  ctx->ty = ty;
  return AF_OK;
}

int32_t af_ctx_get_tile(const af_ctx* ctx) { return ctx ? ctx->ty : -1; }

af_status af_ctx_set_fused_pairs(af_ctx* ctx, int32_t on) {
  if (!ctx) return fail(AF_ERR_ARG, "null ctx");
  if (on != 0 && on != 1) return fail(AF_ERR_ARG, "af_ctx_set_fused_pairs: on must be 0 or 1");
  ctx->fused_pairs = on == 1;
  return AF_OK;
}

int32_t af_ctx_get_fused_pairs(const af_ctx* ctx) { return ctx ? int32_t(ctx->fused_pairs) : -1; }

// ----------------------------------------------------------------- hierarchy

af_status af_hier_create(af_ctx* ctx, int32_t n, const int32_t* level, const int32_t* ix, const int32_t* iy,
                         af_hier** out) {
  if (!ctx || !out || n <= 0 || !level || !ix || !iy) return fail(AF_ERR_ARG, "bad hierarchy arguments");
  auto h = std::make_unique<af_hier>();
  h->ctx = ctx;
  h->pool = ctx->pool;
  h->H.m = ctx->P.m;
  h->H.n0x = ctx->P.n0x;
  h->H.n0y = ctx->P.n0y;
  h->H.lmax = ctx->P.lmax;
  std::vector<Leaf> leaves(n);
  for (int k = 0; k < n; ++k) leaves[k] = {level[k], ix[k], iy[k]};
  const std::string msg = h->H.build(leaves);
  if (!msg.empty()) {
    const bool bal = msg.find("balanced") != std::string::npos || msg.find("cover") != std::string::npos ||
                     msg.find("overlap") != std::string::npos || msg.find("duplicate") != std::string::npos;
    return fail(bal ? AF_ERR_BALANCE : AF_ERR_ARG, "af_hier_create: " + msg);
  }
  h->face_off.assign(h->H.lmax + 2, 0);
  for (int l = 0; l <= h->H.lmax; ++l) {
    h->face_off[l] = int(h->all_faces.size());
    h->all_faces.insert(h->all_faces.end(), h->H.faces[l].begin(), h->H.faces[l].end());
  }
  h->face_off[h->H.lmax + 1] = int(h->all_faces.size());
  // leaves whose eight neighbours are not all leaves of their own level
  h->impure_off.assign(h->H.lmax + 2, 0);
  for (int k = 0; k < n; ++k) {
    const Leaf& L = h->H.leaves[k];
    bool pure = true;
    for (int dy = -1; dy <= 1 && pure; ++dy)
      for (int dx = -1; dx <= 1 && pure; ++dx)
        if ((dx || dy) && h->H.find(L.level, L.ix + dx, L.iy + dy) < 0) pure = false;
    if (!pure) h->impure.push_back(k);
  }
  for (int l = 0, e = 0; l <= h->H.lmax + 1; ++l) {
    while (e < int(h->impure.size()) && h->H.leaves[h->impure[e]].level < l) ++e;
    h->impure_off[l] = e;
  }
  *out = h.release();
  return AF_OK;
}

af_status af_hier_destroy(af_hier* h) {
  if (!h) return AF_OK;
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.second);
  // the tables go back to the pool once no queued work can read them
  if (h->on_device) (void)hipDeviceSynchronize();
  DevPool& pool = *h->pool;
  for (void* p : {static_cast<void*>(h->d_lut), static_cast<void*>(h->d_level), static_cast<void*>(h->d_ix),
                  static_cast<void*>(h->d_iy), static_cast<void*>(h->d_side_mask), static_cast<void*>(h->d_xy),
                  static_cast<void*>(h->d_faces), static_cast<void*>(h->d_nbr), static_cast<void*>(h->d_gnflags),
                  static_cast<void*>(h->d_impure)})
    pool.put(p);
  for (int4* p : h->d_plan) pool.put(p);
  for (uint32_t* p : h->d_plan_flags) pool.put(p);
  for (int4* p : h->d_canon_ops) pool.put(p);
  delete h;
  return AF_OK;
}

int32_t af_hier_num_leaves(const af_hier* h) { return h ? int32_t(h->H.leaves.size()) : -1; }

af_status af_hier_get_leaves(const af_hier* h, int32_t* level, int32_t* ix, int32_t* iy) {
  if (!h || !level || !ix || !iy) return fail(AF_ERR_ARG, "null argument");
  for (size_t k = 0; k < h->H.leaves.size(); ++k) {
    level[k] = h->H.leaves[k].level;
    ix[k] = h->H.leaves[k].ix;
    iy[k] = h->H.leaves[k].iy;
  }
  return AF_OK;
}

af_status af_hier_level_range(const af_hier* h, int32_t level, int32_t* first, int32_t* count) {
  if (!h || !first || !count) return fail(AF_ERR_ARG, "null argument");
  if (level < 0 || level > h->H.lmax) {
    *first = 0;
    *count = 0;
    return AF_OK;
  }
  *count = h->H.level_count[level];
  *first = h->H.level_count[level] ? h->H.level_first[level] : 0;
  return AF_OK;
}

int32_t af_hier_finest_level(const af_hier* h) { return h ? h->H.finest : -1; }

af_status af_hier_side_relations(const af_hier* h, int8_t* rel) {
  if (!h || !rel) return fail(AF_ERR_ARG, "null argument");
  std::memcpy(rel, h->H.rel.data(), h->H.rel.size());
  return AF_OK;
}

const uint8_t* af_hier_side_mask(const af_hier* h) {
  if (!h || hier_device(const_cast<af_hier*>(h)) != AF_OK) return nullptr;
  return h->d_side_mask;
}

const int32_t* af_hier_leaf_xy(const af_hier* h) {
  if (!h || hier_device(const_cast<af_hier*>(h)) != AF_OK) return nullptr;
  return h->d_xy;
}

// ----------------------------------------------------------------- step

// af_patch_step with the choice of where cells outside a patch come from:
// gnx = 0, its ghost layers; gnx > 0, the interiors of its neighbours in the
// complete row-major gnx x gny level that starts at leaf `first` (the
// coarse-step driver on a one-level hierarchy, which then needs no fill).
static af_status patch_step_gather(af_ctx* ctx, const af_state* in, af_state* out, int32_t first, int32_t count,
                                   int32_t level, double dt, double t, int32_t region, double* flux_reg,
                                   const uint8_t* side_mask, const int32_t* leaf_xy, int32_t gnx, int32_t gny,
                                   hipStream_t stream) {
  if (!ctx) return fail(AF_ERR_ARG, "null ctx");
  if (count < 0 || first < 0) return fail(AF_ERR_ARG, "negative patch range");
  if (region != AF_REGION_INTERIOR && region != AF_REGION_LAYER1) return fail(AF_ERR_ARG, "bad region");
  if (level < 0 || level > ctx->P.lmax) return fail(AF_ERR_ARG, "level out of range");
  af_status s = check_state(ctx, in, first + count, "af_patch_step(in)");
  if (s != AF_OK) return s;
  s = check_state(ctx, out, first + count, "af_patch_step(out)");
  if (s != AF_OK) return s;
  if (in->pitch != out->pitch || in->npatch != out->npatch)
    return fail(AF_ERR_LAYOUT, "af_patch_step: in and out differ in layout");
  for (int k = 0; k < 4; ++k)
    if (in->dof[k] == out->dof[k]) return fail(AF_ERR_ARG, "af_patch_step: in and out must be distinct");
  s = check_cfl(ctx, level, dt);
  if (s != AF_OK) return s;
  if ((ctx->P.eq == AF_ROTATION || ctx->P.eq == AF_SWIRL) && !leaf_xy)
    return fail(AF_ERR_ARG, "af_patch_step: rotation and swirl need leaf_xy");
  if (!std::isfinite(t)) return fail(AF_ERR_ARG, "af_patch_step: t must be finite");
  if (count == 0) return AF_OK;
  const double dx = ctx->dx(level), dy = ctx->dy(level);
  StepLaunch L;
  RotParams<float> rp32;
  RotParams<double> rp64;
  SwirlParams<float> sp32;
  SwirlParams<double> sp64;
  BurgersParams<float> bp32;
  BurgersParams<double> bp64;
  L.fp32 = ctx->fp32();
  L.eq = ctx->P.eq;
  L.m = ctx->P.m;
  L.ty = ctx->ty;
  for (int k = 0; k < 4; ++k) {
    L.in[k] = in->dof[k];
    L.out[k] = out->dof[k];
  }
  L.npatch = in->npatch;
  L.pitch = in->pitch;
  L.first = first;
  L.count = count;
  L.region = region;
  L.dtdx = dt / dx;
  L.dtdy = dt / dy;
  L.a = ctx->P.a;
  L.b = ctx->P.b;
  L.c = ctx->P.c;
  L.len_dt_x = dy * dt;
  L.len_dt_y = dx * dt;
  L.reg = flux_reg;
  L.side_mask = flux_reg ? side_mask : nullptr;
  L.leaf_xy = leaf_xy;
  L.gnx = gnx;
  L.gny = gny;
  if (ctx->P.eq == AF_ROTATION) {
    // the rotation angle depends on dt itself, not on dt/dx: no cache
    const double th[2] = {ctx->P.omega * 0.5 * dt, ctx->P.omega * dt};
    for (int t = 0; t < 2; ++t) {
      rp64.cs[t] = std::cos(th[t]);
      rp64.sn[t] = std::sin(th[t]);
    }
    rp64.x0 = ctx->P.x0; rp64.y0 = ctx->P.y0; rp64.dx = dx; rp64.dy = dy;
    rp64.omega = ctx->P.omega; rp64.xc = ctx->P.xc; rp64.yc = ctx->P.yc;
    rp32.cs[0] = float(rp64.cs[0]); rp32.cs[1] = float(rp64.cs[1]);
    rp32.sn[0] = float(rp64.sn[0]); rp32.sn[1] = float(rp64.sn[1]);
    rp32.x0 = float(rp64.x0); rp32.y0 = float(rp64.y0); rp32.dx = float(dx); rp32.dy = float(dy);
    rp32.omega = float(rp64.omega); rp32.xc = float(rp64.xc); rp32.yc = float(rp64.yc);
    L.weights = ctx->fp32() ? static_cast<const void*>(&rp32) : static_cast<const void*>(&rp64);
  } else if (ctx->P.eq == AF_SWIRL) {
    // cos(pi s) at every time the step needs, formed as the traces form them
    // (t + tau, then stage offsets -tau/2, -tau)
    constexpr double kPi = 3.14159265358979323846264338327950288;
    const double tau[2] = {0.5 * dt, dt};
    for (int k = 0; k < 2; ++k) {
      const double t1 = t + tau[k], hh = -tau[k];
      sp64.tau[k] = tau[k];
      sp64.cos_rk[k][0] = std::cos(kPi * t1);
      sp64.cos_rk[k][1] = std::cos(kPi * (t1 + 0.5 * hh));
      sp64.cos_rk[k][2] = std::cos(kPi * (t1 + hh));
    }
    for (int k = 0; k < 3; ++k) sp64.cos_fx[k] = std::cos(kPi * (t + 0.5 * k * dt));
    sp64.x0 = ctx->P.x0; sp64.y0 = ctx->P.y0; sp64.dx = dx; sp64.dy = dy;
    sp64.kx = std::sin(kPi * dx) / (kPi * dx);
    sp64.ky = std::sin(kPi * dy) / (kPi * dy);
    sp32.x0 = float(sp64.x0); sp32.y0 = float(sp64.y0); sp32.dx = float(dx); sp32.dy = float(dy);
    sp32.kx = float(sp64.kx); sp32.ky = float(sp64.ky);
    for (int k = 0; k < 2; ++k) {
      sp32.tau[k] = float(sp64.tau[k]);
      for (int q = 0; q < 3; ++q) sp32.cos_rk[k][q] = float(sp64.cos_rk[k][q]);
    }
    for (int k = 0; k < 3; ++k) sp32.cos_fx[k] = float(sp64.cos_fx[k]);
    L.weights = ctx->fp32() ? static_cast<const void*>(&sp32) : static_cast<const void*>(&sp64);
  } else if (ctx->P.eq == AF_BURGERS) {
    for (int k = 0; k < 2; ++k) {
      const double tau = (k + 1) * 0.5 * dt;
      bp64.tdx[k] = tau / dx;
      bp64.tdy[k] = tau / dy;
      bp32.tdx[k] = float(bp64.tdx[k]);
      bp32.tdy[k] = float(bp64.tdy[k]);
    }
    L.weights = ctx->fp32() ? static_cast<const void*>(&bp32) : static_cast<const void*>(&bp64);
  } else {
    L.weights = weights_for(ctx, dt / dx, dt / dy);
    if (!L.weights) return fail(AF_ERR_STATE, "acoustic stencils lack their mirror symmetry");
  }
  AF_HIP(launch_patch_step(L, stream));
  return AF_OK;
}

af_status af_patch_step(af_ctx* ctx, const af_state* in, af_state* out, int32_t first, int32_t count,
                        int32_t level, double dt, double t, int32_t region, double* flux_reg,
                        const uint8_t* side_mask, const int32_t* leaf_xy, hipStream_t stream) {
  return patch_step_gather(ctx, in, out, first, count, level, dt, t, region, flux_reg, side_mask, leaf_xy, 0, 0,
                           stream);
}

// ----------------------------------------------------------------- fill etc.

namespace {

// The fill plan of hierarchy h for sources of level >= smin (smin <= lmax),
// resolved on the device on first use.  The plan depends on the leaf set and
// m only, so it serves every buffer pair and every lower target bound.
af_status fill_plan(af_ctx* ctx, af_hier* h, int smin, hipStream_t stream) {
  if (int(h->d_plan.size()) <= h->H.lmax) {
    h->d_plan.resize(h->H.lmax + 1, nullptr);
    h->d_plan_flags.resize(h->H.lmax + 1, nullptr);
    h->d_canon_ops.resize(h->H.lmax + 1, nullptr);
  }
  if (h->d_plan[smin]) return AF_OK;
  af_status s;
  if ((s = ctx_device(ctx)) != AF_OK || (s = hier_device(h)) != AF_OK) return s;
  const size_t n = h->H.leaves.size();
  int4* plan = nullptr;
  uint32_t* flags = nullptr;
  DevPool& pool = *h->pool;
  AF_HIP(pool.get(reinterpret_cast<void**>(&plan), std::max<size_t>(1, n * size_t(ctx->nentries)) * sizeof(int4)));
  if (pool.get(reinterpret_cast<void**>(&flags), std::max<size_t>(1, n) * sizeof(uint32_t)) != hipSuccess) {
    pool.put(plan);
    return fail(AF_ERR_DEVICE, "fill plan allocation");
  }
  h->d_plan[smin] = plan;
  h->d_plan_flags[smin] = flags;
  if (smin == 0) {
    AF_HIP(pool.get(reinterpret_cast<void**>(&h->d_nbr), std::max<size_t>(1, n) * 9 * sizeof(int32_t)));
    AF_HIP(pool.get(reinterpret_cast<void**>(&h->d_gnflags), std::max<size_t>(1, n) * sizeof(uint32_t)));
  }
  AF_HIP(launch_fill_plan(h->dev, ctx->d_entries, ctx->nentries, ctx->P.m, smin, plan, flags,
                          smin == 0 ? h->d_nbr : nullptr, smin == 0 ? h->d_gnflags : nullptr, stream));
  // the batched step's vertex copies for this bound, resolved from the plan
  const int ncanon = int(h->impure.size()) - h->impure_off[smin];
  const int nbnd = int(ctx->h_bnd.size());
  if (ncanon > 0 && nbnd > 0) {
    int4* ops = nullptr;
    AF_HIP(pool.get(reinterpret_cast<void**>(&ops), size_t(ncanon) * nbnd * sizeof(int4)));
    h->d_canon_ops[smin] = ops;
    AF_HIP(launch_canon_ops(plan, ctx->d_entries, ctx->nentries, ctx->d_bnd, nbnd, h->d_impure + h->impure_off[smin],
                            ncanon, h->d_level, ops, stream));
  }
  return AF_OK;
}

}  // namespace

af_status af_ghost_fill(af_ctx* ctx, const af_hier* hc, af_state* bufs, uint32_t mask, int32_t tmin, int32_t smin,
                        hipStream_t stream) {
  if (!ctx || !hc) return fail(AF_ERR_ARG, "null argument");
  af_hier* h = const_cast<af_hier*>(hc);
  af_status s = check_pair(ctx, h, bufs, "af_ghost_fill");
  if (s != AF_OK) return s;
  if (tmin < 0 || smin < 0) return fail(AF_ERR_ARG, "negative level bound");
  if (smin > h->H.lmax) return AF_OK;  // no level may serve as a source
  int first = -1;
  for (int l = tmin; l <= h->H.lmax && first < 0; ++l)
    if (h->H.level_count[l]) first = h->H.level_first[l];
  if (first < 0) return AF_OK;
  if ((s = fill_plan(ctx, h, smin, stream)) != AF_OK) return s;
  // the coarse->fine phase is needed only if some target level has leaves
  // one level down that may serve as sources
  bool need_b = false;
  for (int l = std::max(tmin, 1); l <= h->H.lmax; ++l)
    if (h->H.level_count[l] && h->H.level_count[l - 1] && l - 1 >= smin) need_b = true;
  const int n = int(h->H.leaves.size()) - first;
  const BufLaunch b = make_buf(ctx, &bufs[0], &bufs[1], mask);
  for (int phase = 0; phase < (need_b ? 2 : 1); ++phase)
    AF_HIP(launch_fill_apply(ctx->fp32(), b, h->dev, ctx->d_entries, ctx->nentries, h->d_plan[smin],
                             h->d_plan_flags[smin], ctx->d_fillw, first, n, phase, stream));
  return AF_OK;
}

af_status af_flux_correct(af_ctx* ctx, const af_hier* h, af_state* bufs, uint32_t mask, int32_t level,
                          double* flux_reg, hipStream_t stream) {
  if (!ctx || !h || !flux_reg) return fail(AF_ERR_ARG, "null argument");
  af_status s = check_pair(ctx, h, bufs, "af_flux_correct");
  if (s != AF_OK) return s;
  if (level < 0 || level > h->H.lmax) return fail(AF_ERR_ARG, "level out of range");
  if ((s = hier_device(const_cast<af_hier*>(h))) != AF_OK) return s;
  const int off = h->face_off[level], nf = h->face_off[level + 1] - off;
  const double inv_area = 1.0 / (ctx->dx(level) * ctx->dy(level));
  AF_HIP(launch_flux_correct(ctx->fp32(), make_buf(ctx, &bufs[0], &bufs[1], mask), h->d_faces + off, nf, flux_reg,
                             level, inv_area, stream));
  return AF_OK;
}

af_status af_regrid_tag(af_ctx* ctx, const af_hier* h, const af_state* bufs, uint32_t mask, int32_t mode,
                        int32_t comp, double theta_r, double theta_c, int8_t* tags, double* values,
                        hipStream_t stream) {
  if (!ctx || !h || !tags) return fail(AF_ERR_ARG, "null argument");
  af_status s = check_pair(ctx, h, bufs, "af_regrid_tag");
  if (s != AF_OK) return s;
  if (mode != AF_TAG_GRADIENT && mode != AF_TAG_MAXMIN) return fail(AF_ERR_ARG, "bad tag mode");
  if (comp < 0 || comp >= ctx->ncomp) return fail(AF_ERR_ARG, "component out of range");
  if ((s = hier_device(const_cast<af_hier*>(h))) != AF_OK) return s;
  AF_HIP(launch_tag(ctx->fp32(), make_buf(ctx, &bufs[0], &bufs[1], mask), h->dev, mode, comp,
                    1.0 / (2.0 * ctx->dx(0)), 1.0 / (2.0 * ctx->dy(0)), theta_r, theta_c, tags, values, stream));
  return AF_OK;
}

af_status af_hier_regrid(af_ctx* ctx, const af_hier* old, const int8_t* tags, af_hier** out) {
  if (!ctx || !old || !tags || !out) return fail(AF_ERR_ARG, "null argument");
  const std::vector<Leaf> nl = old->H.regrid(tags);
  std::vector<int32_t> lv(nl.size()), vx(nl.size()), vy(nl.size());
  for (size_t k = 0; k < nl.size(); ++k) {
    lv[k] = nl[k].level;
    vx[k] = nl[k].ix;
    vy[k] = nl[k].iy;
  }
  return af_hier_create(ctx, int32_t(nl.size()), lv.data(), vx.data(), vy.data(), out);
}

af_status af_regrid_apply(af_ctx* ctx, const af_hier* old, const af_state* old_bufs, uint32_t old_mask,
                          const af_hier* nh, af_state* dst, hipStream_t stream) {
  if (!ctx || !old || !nh || !dst) return fail(AF_ERR_ARG, "null argument");
  af_status s = check_pair(ctx, old, old_bufs, "af_regrid_apply(old)");
  if (s != AF_OK) return s;
  s = check_state(ctx, dst, int(nh->H.leaves.size()), "af_regrid_apply(dst)");
  if (s != AF_OK) return s;
  if (dst->pitch != old_bufs[0].pitch) return fail(AF_ERR_LAYOUT, "af_regrid_apply: pitch differs");
  for (int k = 0; k < 4; ++k)
    if (dst->dof[k] == old_bufs[0].dof[k] || dst->dof[k] == old_bufs[1].dof[k])
      return fail(AF_ERR_ARG, "af_regrid_apply: dst must differ from the old buffers");
  std::vector<Transfer> tr(nh->H.leaves.size());
  for (size_t k = 0; k < nh->H.leaves.size(); ++k) {
    const Leaf& L = nh->H.leaves[k];
    Transfer& X = tr[k];
    X.qx = X.qy = 0;
    for (int q = 0; q < 4; ++q) X.src[q] = -1;
    const int same = old->H.find(L.level, L.ix, L.iy);
    if (same >= 0) {
      X.mode = 0;
      X.src[0] = same;
      continue;
    }
    const int par = L.level > 0 ? old->H.find(L.level - 1, L.ix >> 1, L.iy >> 1) : -1;
    if (par >= 0) {
      X.mode = 1;
      X.src[0] = par;
      X.qx = L.ix & 1;
      X.qy = L.iy & 1;
      continue;
    }
    X.mode = 2;
    for (int q = 0; q < 4; ++q) {
      X.src[q] = old->H.find(L.level + 1, 2 * L.ix + (q & 1), 2 * L.iy + (q >> 1));
      if (X.src[q] < 0) return fail(AF_ERR_STATE, "af_regrid_apply: new leaf is not a copy, child or parent of old leaves");
    }
  }
  if ((s = hier_device(const_cast<af_hier*>(old))) != AF_OK) return s;
  hipError_t err;
  Transfer* d_tr = pool_upload(*ctx->pool, tr, &err);
  if (err != hipSuccess) return fail(AF_ERR_DEVICE, "transfer table upload");
  HierDev HO = old->dev;
  BufLaunch ob = make_buf(ctx, &old_bufs[0], &old_bufs[1], old_mask);
  BufLaunch nb = make_buf(ctx, dst, dst, 0);
  err = launch_transfer(ctx->fp32(), ob, HO, nb, d_tr, int(tr.size()), stream);
  if (err == hipSuccess) err = hipStreamSynchronize(stream);
  if (err == hipSuccess) ctx->pool->put(d_tr);  // after a failure the block stays out of the pool
  if (err != hipSuccess) return fail(AF_ERR_DEVICE, std::string("transfer: ") + hipGetErrorString(err));
  // the new hierarchy's ghost-fill plans, so that its first coarse step
  // does not resolve them
  af_hier* nhm = const_cast<af_hier*>(nh);
  for (int l = 0; l <= nhm->H.finest; ++l)
    if ((s = fill_plan(ctx, nhm, l, stream)) != AF_OK) return s;
  return AF_OK;
}

af_status af_reduce_sum(af_ctx* ctx, const af_hier* h, const af_state* bufs, uint32_t mask, double* out,
                        hipStream_t stream) {
  if (!ctx || !h || !out) return fail(AF_ERR_ARG, "null argument");
  af_status s = check_pair(ctx, h, bufs, "af_reduce_sum");
  if (s != AF_OK) return s;
  if ((s = hier_device(const_cast<af_hier*>(h))) != AF_OK) return s;
  const int n = int(h->H.leaves.size());
  if (ctx->part_cap < n * ctx->ncomp) {
    (void)hipFree(ctx->d_part);
    ctx->d_part = nullptr;
    AF_HIP(hipMalloc(&ctx->d_part, size_t(n) * ctx->ncomp * sizeof(double)));
    ctx->part_cap = n * ctx->ncomp;
  }
  AF_HIP(launch_sum(ctx->fp32(), make_buf(ctx, &bufs[0], &bufs[1], mask), h->dev, ctx->dx(0) * ctx->dy(0),
                    ctx->d_part, out, stream));
  return AF_OK;
}

af_status af_reduce_sum_noalloc(af_ctx* ctx, const af_hier* h, const af_state* bufs, uint32_t mask, double* out,
                                hipStream_t stream) {
  if (!ctx || !h || !out) return fail(AF_ERR_ARG, "null argument");
  af_status s = check_pair(ctx, h, bufs, "af_reduce_sum_noalloc");
  if (s != AF_OK) return s;
  const size_t need = h->H.leaves.size() * size_t(ctx->ncomp);
  if (need > kScratchSums)
    return fail(AF_ERR_ARG, "af_reduce_sum_noalloc: nleaves * ncomp = " + std::to_string(need) +
                                " exceeds the static scratch of " + std::to_string(kScratchSums) + " partial sums");
  // the hierarchy's tables must already be on the device: uploading them
  // would allocate
  if (!h->on_device)
    return fail(AF_ERR_STATE,
                "af_reduce_sum_noalloc: the hierarchy's device tables are not uploaded yet (any launching call with "
                "it, or af_hier_leaf_xy, uploads them)");
  double* part = nullptr;
  AF_HIP(scratch_sums(&part));
  AF_HIP(launch_sum(ctx->fp32(), make_buf(ctx, &bufs[0], &bufs[1], mask), h->dev, ctx->dx(0) * ctx->dy(0), part, out,
                    stream));
  return AF_OK;
}

// ----------------------------------------------------------------- level advance

namespace {

// A level the level advance can run on: it covers the periodic domain (every
// patch has its eight neighbours on it), so its leaves are the complete
// row-major nx x ny array of the level and neighbours are found by index.
af_status level_grid(af_hier* h, int level, int* nx, int* ny) {
  if (h->nbr_ok.empty()) h->nbr_ok.assign(h->H.lmax + 1, -1);
  *nx = h->H.n0x << level;
  *ny = h->H.n0y << level;
  if (h->nbr_ok[level] < 0) {
    const int first = h->H.level_count[level] ? h->H.level_first[level] : 0;
    const int count = h->H.level_count[level];
    int ok = count == *nx * *ny;
    for (int k = 0; k < count && ok; ++k) {
      const Leaf& L = h->H.leaves[first + k];
      ok = L.level == level && L.ix == k % *nx && L.iy == k / *nx;
    }
    h->nbr_ok[level] = ok;
  }
  if (!h->nbr_ok[level])
    return fail(AF_ERR_STATE, "af_level_advance: a patch of this level has a neighbour on another level");
  return AF_OK;
}

// The shape set on the context if it runs here (up: the weights have the
// upwind pattern), else the largest K with the smallest block.
void default_advance_shape(const af_ctx* c, bool up, int* k, int* nt) {
  int ks[32], nts[32];
  const int n = level_advance_shapes(c->fp32(), c->P.eq, c->P.m, ks, nts, 32, up);
  *k = 0;
  *nt = 0;
  if (c->adv_k) {
    for (int i = 0; i < n; ++i)
      if (ks[i] == c->adv_k && nts[i] == c->adv_nt) { *k = ks[i]; *nt = nts[i]; return; }
  }
  // default: the largest K with the smallest block
  for (int i = 0; i < n; ++i)
    if (ks[i] > *k || (ks[i] == *k && nts[i] < *nt)) { *k = ks[i]; *nt = nts[i]; }
}

}  // namespace

af_status af_ctx_set_advance_shape(af_ctx* ctx, int32_t k, int32_t nt) {
  if (!ctx) return fail(AF_ERR_ARG, "null ctx");
  int ks[32], nts[32];
  const int n = level_advance_shapes(ctx->fp32(), ctx->P.eq, ctx->P.m, ks, nts, 32, true);
  for (int i = 0; i < n; ++i)
    if (ks[i] == k && nts[i] == nt) {
      ctx->adv_k = k;
      ctx->adv_nt = nt;
      return AF_OK;
    }
  return fail(AF_ERR_ARG, "unsupported level-advance shape for this problem");
}

af_status af_ctx_get_advance_shape(const af_ctx* ctx, int32_t* k, int32_t* nt) {
  if (!ctx || !k || !nt) return fail(AF_ERR_ARG, "null argument");
  int kk, nn;
  // the upwind pattern needs both velocity components positive (and small
  // enough time steps)
  default_advance_shape(ctx, ctx->P.eq == AF_ADVECTION && ctx->P.a > 0 && ctx->P.b > 0, &kk, &nn);
  *k = kk;
  *nt = nn;
  return AF_OK;
}

int32_t af_ctx_advance_shapes(const af_ctx* ctx, int32_t* ks, int32_t* nts, int32_t cap) {
  if (!ctx) return -1;
  int k2[32], n2[32];
  const int n = level_advance_shapes(ctx->fp32(), ctx->P.eq, ctx->P.m, k2, n2, 32, true);
  for (int i = 0; i < n && i < cap; ++i) {
    if (ks) ks[i] = k2[i];
    if (nts) nts[i] = n2[i];
  }
  return n;
}

int32_t af_ctx_advance_shapes_upwind(const af_ctx* ctx, int32_t* ks, int32_t* nts, int32_t cap) {
  if (!ctx) return -1;
  int k2[32], n2[32];
  // the list with the upwind-only shapes holds the two-pass shapes first
  const int two = level_advance_shapes(ctx->fp32(), ctx->P.eq, ctx->P.m, k2, n2, 32, false);
  const int all = level_advance_shapes(ctx->fp32(), ctx->P.eq, ctx->P.m, k2, n2, 32, true);
  for (int i = two; i < all && i - two < cap; ++i) {
    if (ks) ks[i - two] = k2[i];
    if (nts) nts[i - two] = n2[i];
  }
  return all - two;
}

af_status af_level_advance(af_ctx* ctx, af_hier* h, af_state* bufs, uint32_t* mask, int32_t level, double dt,
                           int32_t nsteps, hipStream_t stream) {
  if (!ctx || !h || !mask) return fail(AF_ERR_ARG, "null argument");
  af_status s = check_pair(ctx, h, bufs, "af_level_advance");
  if (s != AF_OK) return s;
  if (level < 0 || level > h->H.lmax) return fail(AF_ERR_ARG, "level out of range");
  if (nsteps < 0) return fail(AF_ERR_ARG, "negative step count");
  for (int k = 0; k < 4; ++k)
    if (bufs[0].dof[k] == bufs[1].dof[k]) return fail(AF_ERR_ARG, "af_level_advance: the two buffers must differ");
  if ((s = check_cfl(ctx, level, dt)) != AF_OK) return s;
  const int count = h->H.level_count[level];
  if (count == 0 || nsteps == 0) return AF_OK;
  const int first = h->H.level_first[level];
  int nx, ny;
  if ((s = level_grid(h, level, &nx, &ny)) != AF_OK) return s;
  const double dx = ctx->dx(level), dy = ctx->dy(level);
  AdvanceLaunch L;
  L.fp32 = ctx->fp32();
  L.eq = ctx->P.eq;
  L.m = ctx->P.m;
  L.npatch = bufs[0].npatch;
  L.pitch = bufs[0].pitch;
  L.first = first;
  L.count = count;
  L.nx = nx;
  L.ny = ny;
  L.dtdx = dt / dx;
  L.dtdy = dt / dy;
  L.a = ctx->P.a;
  L.b = ctx->P.b;
  L.c = ctx->P.c;
  L.weights = weights_for(ctx, dt / dx, dt / dy);
  if (!L.weights) return fail(AF_ERR_STATE, "acoustic stencils lack their mirror symmetry");
  const bool up = level_advance_up_pattern(L.fp32, L.eq, L.weights);
  int K, NT;
  default_advance_shape(ctx, up, &K, &NT);
  if (K == 0) return fail(AF_ERR_ARG, "no level-advance kernel for this (precision, equation, m)");
  int done = 0;
  while (done < nsteps) {
    // a tail shorter than K runs with the K = 1 (or 2) kernel of the same family
    int kk = K, nt = NT;
    if (nsteps - done < K) {
      int ks[32], nts[32];
      const int n = level_advance_shapes(ctx->fp32(), ctx->P.eq, ctx->P.m, ks, nts, 32, up);
      kk = 0;
      for (int i = 0; i < n; ++i)
        if (ks[i] <= nsteps - done && (ks[i] > kk || (ks[i] == kk && nts[i] < nt))) { kk = ks[i]; nt = nts[i]; }
      if (kk == 0) return fail(AF_ERR_STATE, "no level-advance kernel short enough for the remaining steps");
    }
    L.k = kk;
    L.nt = nt;
    const int cur = (*mask >> level) & 1;
    for (int k = 0; k < 4; ++k) {
      L.in[k] = bufs[cur].dof[k];
      L.out[k] = bufs[cur ^ 1].dof[k];
    }
    AF_HIP(launch_level_advance(L, stream));
    *mask ^= (1u << level);
    done += kk;
  }
  return AF_OK;
}

// ----------------------------------------------------------------- tagger access

struct AfTagView {
  bool fp32;
  int ncomp, m, npatch, pitch, lmax, nleaves;
  const void* dof0[4];
  const void* dof1[4];
  const int32_t* plevel;
};

af_status af_internal_tag_view(const af_ctx* ctx, const af_hier* h, const af_state* bufs, AfTagView* v) {
  if (!ctx || !h || !v) return fail(AF_ERR_ARG, "null argument");
  af_status s = check_pair(ctx, h, bufs, "tag view");
  if (s != AF_OK) return s;
  if ((s = hier_device(const_cast<af_hier*>(h))) != AF_OK) return s;
  v->fp32 = ctx->fp32();
  v->ncomp = ctx->ncomp;
  v->m = ctx->P.m;
  v->npatch = bufs[0].npatch;
  v->pitch = bufs[0].pitch;
  v->lmax = ctx->P.lmax;
  v->nleaves = int(h->H.leaves.size());
  for (int k = 0; k < 4; ++k) {
    v->dof0[k] = bufs[0].dof[k];
    v->dof1[k] = bufs[1].dof[k];
  }
  v->plevel = h->d_level;
  return AF_OK;
}

// ----------------------------------------------------------------- autotuner

af_status af_autotune(af_ctx* ctx, af_hier* h, af_state* bufs, int32_t level, double dt, int32_t reps,
                      double* best_step_us, double* best_advance_us, hipStream_t stream) {
  if (!ctx || !h) return fail(AF_ERR_ARG, "null argument");
  af_status s = check_pair(ctx, h, bufs, "af_autotune");
  if (s != AF_OK) return s;
  if (reps < 1) return fail(AF_ERR_ARG, "reps must be >= 1");
  if ((s = hier_device(h)) != AF_OK) return s;
  const int count = level >= 0 && level <= h->H.lmax ? h->H.level_count[level] : 0;
  if (count == 0) return fail(AF_ERR_ARG, "level has no leaves");
  const int first = h->H.level_first[level];
  hipEvent_t e0, e1;
  AF_HIP(hipEventCreate(&e0));
  AF_HIP(hipEventCreate(&e1));
  auto timed = [&](auto&& body, double* us) -> af_status {
    af_status st = body();  // warm-up launch
    if (st != AF_OK) return st;
    if (hipEventRecord(e0, stream) != hipSuccess) return fail(AF_ERR_DEVICE, "event record");
    for (int r = 0; r < reps; ++r)
      if ((st = body()) != AF_OK) return st;
    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return fail(AF_ERR_DEVICE, "event sync");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *us = 1e3 * double(ms) / reps;
    return AF_OK;
  };
  // patch-step tile height
  double best = 1e300;
  int best_ty = ctx->ty;
  const int tys[5] = {2, 4, 8, 16, 32};
  for (int ty : tys) {
    if (!step_shape_supported(ctx->P.m, ty)) continue;
    ctx->ty = ty;
    double us;
    s = timed([&]() {
          return af_patch_step(ctx, &bufs[0], &bufs[1], first, count, level, dt, 0.0, 0, nullptr, nullptr, h->d_xy,
                               stream);
        },
              &us);
    if (s != AF_OK) break;
    if (us < best) { best = us; best_ty = ty; }
  }
  ctx->ty = best_ty;
  if (best_step_us) *best_step_us = best;
  // level-advance shape (per step), if the level allows it
  double best_adv = -1.0;
  int gnx, gny;
  if (s == AF_OK && level_grid(h, level, &gnx, &gny) == AF_OK) {
    int ks[32], nts[32];
    const bool up = level_advance_up_pattern(ctx->fp32(), ctx->P.eq,
                                             weights_for(ctx, dt / ctx->dx(level), dt / ctx->dy(level)));
    const int n = level_advance_shapes(ctx->fp32(), ctx->P.eq, ctx->P.m, ks, nts, 32, up);
    double b2 = 1e300;
    int bk = 0, bn = 0;
    for (int i = 0; i < n; ++i) {
      ctx->adv_k = ks[i];
      ctx->adv_nt = nts[i];
      uint32_t mk = 0;
      double us;
      s = timed([&]() { return af_level_advance(ctx, h, bufs, &mk, level, dt, ks[i], stream); }, &us);
      if (s != AF_OK) break;
      us /= ks[i];
      if (us < b2) { b2 = us; bk = ks[i]; bn = nts[i]; }
    }
    ctx->adv_k = bk;
    ctx->adv_nt = bn;
    if (bk > 0) best_adv = b2;  // stays -1 when no shape is compiled for (precision, equation, m)
  }
  g_err.clear();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_advance_us) *best_advance_us = best_adv;
  return s;
}

// ----------------------------------------------------------------- AMR driver

namespace {

struct Driver {
  af_ctx* ctx;
  af_hier* h;
  af_state* bufs;
  uint32_t mask;
  double* reg;
  hipStream_t st;
  // > 0: the hierarchy is one complete level (gnx x gny patches); steps read
  // neighbours' interiors and no fill is needed
  int gnx = 0, gny = 0;

  af_status step_level(int l, double t, double dt, int region) {
    int first, count;
    af_hier_level_range(h, l, &first, &count);
    const int cur = (mask >> l) & 1;
    // an empty level still flips, so that the mask after a coarse step is
    // always "bit 0 flipped" (subcycled) or "bits 0..finest flipped" (global)
    mask ^= (1u << l);
    if (count == 0) return AF_OK;
    return patch_step_gather(ctx, &bufs[cur], &bufs[cur ^ 1], first, count, l, dt, t, region, reg,
                             h->d_side_mask, h->d_xy, gnx, gny, st);
  }

  af_status advance(int l, double t, double dt, bool first_of_pair, int finest) {
    af_status s = step_level(l, t, dt, (l > 0 && first_of_pair) ? AF_REGION_LAYER1 : AF_REGION_INTERIOR);
    if (s != AF_OK) return s;
    if (l + 1 <= finest) {
      if ((s = advance(l + 1, t, 0.5 * dt, true, finest)) != AF_OK) return s;
      if ((s = af_ghost_fill(ctx, h, bufs, mask, l + 1, l + 1, st)) != AF_OK) return s;
      if ((s = advance(l + 1, t + 0.5 * dt, 0.5 * dt, false, finest)) != AF_OK) return s;
      int first, count;
      af_hier_level_range(h, l, &first, &count);
      if (count) {
        if ((s = af_flux_correct(ctx, h, bufs, mask, l, reg, st)) != AF_OK) return s;
      }
    }
    return AF_OK;
  }

  // ---- batched coarse step (constant coefficients, Sec. 3.2): one launch
  // per substep start time for all levels that start a step then, with the
  // ghost data staged from the fill plans; before it, one launch for the
  // conservative fix of the levels that just completed a pair and the
  // fill's vertex copies on coarse-fine lines.
  af_status sync(int smin, int fix_lo, int fix_hi) {
    const int F = h->H.finest;
    AmrSyncLaunch S{};
    S.fp32 = ctx->fp32();
    S.b = make_buf(ctx, &bufs[0], &bufs[1], mask);
    S.plevel = h->d_level;
    S.reg = reg;
    S.inv_area0 = 1.0 / (ctx->dx(0) * ctx->dy(0));
    if (smin >= 0 && smin <= F && h->d_canon_ops[smin]) {
      S.cops = h->d_canon_ops[smin];
      S.ncops = (int(h->impure.size()) - h->impure_off[smin]) * int(ctx->h_bnd.size());
    }
    if (fix_lo <= fix_hi) {
      const int off = h->face_off[fix_lo];
      S.faces = h->d_faces + off;
      S.nfaces = h->face_off[fix_hi + 1] - off;
    }
    AF_HIP(launch_amr_sync(S, st));
    return AF_OK;
  }

  af_status batched_step(int tau, int l0) {
    const int F = h->H.finest;
    // the batched step addresses a DOF array with 32-bit element offsets
    if (double(bufs[0].npatch) * (ctx->P.m + 5) * bufs[0].pitch * ctx->ncomp >= 2147483648.0)
      return fail(AF_ERR_LAYOUT, "af_amr_coarse_step: a DOF array of 2^31 or more elements");
    const double dt0 = dt0_;
    AmrStepLaunch L{};
    L.fp32 = ctx->fp32();
    L.eq = ctx->P.eq;
    L.m = ctx->P.m;
    L.ty = ctx->ty;
    for (int b = 0; b < 2; ++b)
      for (int k = 0; k < 4; ++k) L.p[b][k] = bufs[b].dof[k];
    L.npatch = bufs[0].npatch;
    L.pitch = bufs[0].pitch;
    L.mask = mask;
    L.lev0 = l0;
    L.nlev = F - l0 + 1;
    for (int k = 0; k < L.nlev; ++k) {
      const int l = l0 + k;
      const double dtl = dt0 / double(1 << l);
      L.count[k] = h->H.level_count[l];
      L.first[k] = L.count[k] ? h->H.level_first[l] : 0;
      // the first of a pair of fine substeps also advances ghost layer 1
      L.region[k] = (l > 0 && ((tau >> (F - l)) & 1) == 0) ? AF_REGION_LAYER1 : AF_REGION_INTERIOR;
      L.len_dt_x[k] = ctx->dy(l) * dtl;
      L.len_dt_y[k] = ctx->dx(l) * dtl;
      mask ^= (1u << l);  // an empty level flips too (the mask convention of a coarse step)
    }
    L.dtdx = dt0 / ctx->dx(0);
    L.dtdy = dt0 / ctx->dy(0);
    L.a = ctx->P.a;
    L.b = ctx->P.b;
    L.c = ctx->P.c;
    L.reg = reg;
    L.side_mask = h->d_side_mask;
    L.plan = h->d_plan[l0];
    L.entries = ctx->d_entries;
    L.nentries = ctx->nentries;
    L.ninner = ctx->ninner;
    L.fw = ctx->d_fillw;
    L.nbr = h->d_nbr;
    L.gnflags = h->d_gnflags;
    L.weights = weights_for(ctx, L.dtdx, L.dtdy);
    if (!L.weights) return fail(AF_ERR_STATE, "acoustic stencils lack their mirror symmetry");
    if (ctx->P.eq == AF_ACOUSTICS && !(L.weights_dev = weights_dev_for(ctx, L.dtdx, L.dtdy)))
      return fail(AF_ERR_DEVICE, "acoustic weight upload failed");
    L.pair = pair_;  // level F (the last here, region layer 1 at even tau) takes its pair
    const bool timed = ev && nev < max_ev;
    if (timed) AF_HIP(hipEventRecord(ev[2 * nev], st));
    AF_HIP(launch_amr_step(L, st));
    if (timed) {
      AF_HIP(hipEventRecord(ev[2 * nev + 1], st));
      if (ev_cells) {
        double cells = 0.0;
        for (int k = 0; k < L.nlev; ++k)
          cells += double(L.count[k]) * ctx->P.m * ctx->P.m * (L.pair && k == L.nlev - 1 ? 2 : 1);
        ev_cells[nev] = cells;
      }
      ++nev;
    }
    return AF_OK;
  }

  // measurement (af_amr_coarse_step_timed): event pairs around the step
  // launches of the batched path
  hipEvent_t* ev = nullptr;
  double* ev_cells = nullptr;
  int max_ev = 0, nev = 0;

  double dt0_ = 0.0;
  bool pair_ = false;
  // several coarse steps in one call (af_amr_coarse_steps): the last launch
  // of a step, the fix of levels 0..F-1, joins the first launch of the next
  // (vertex copies only), which touches nodes only
  bool defer_fix = false;    // leave this step's final fix to the next step
  bool pending_fix = false;  // the previous step's final fix is still to make

  af_status coarse_step_batched(double dt0) {
    const int F = h->H.finest;
    dt0_ = dt0;
    af_status s;
    for (int l = 0; l <= F; ++l)
      if ((s = fill_plan(ctx, h, l, st)) != AF_OK) return s;
    // fused pairs: the launch of each even time point also takes the finest
    // level's second substep, so the odd time points (where only level F
    // starts a step) need no launch
    pair_ = ctx->fused_pairs && F >= 2 && amr_pair_supported(ctx->P.m);
    for (int tau = 0; tau < (1 << F); tau += pair_ ? 2 : 1) {
      // the coarsest level that starts a step at tau
      const int l0 = tau == 0 ? 0 : F - __builtin_ctz(unsigned(tau));
      if (tau == 0) {
        if ((s = pending_fix ? sync(0, 0, F - 1) : sync(0, 1, 0)) != AF_OK) return s;
        pending_fix = false;
      } else if (l0 < F) {
        if ((s = sync(l0, l0, F - 1)) != AF_OK) return s;
      }
      if ((s = batched_step(tau, l0)) != AF_OK) return s;
    }
    if (F > 0 && defer_fix) {
      pending_fix = true;
      return AF_OK;
    }
    return F > 0 ? sync(-1, 0, F - 1) : AF_OK;
  }

  af_status coarse_step(double t0, double dt0) {
    if (!gnx && (ctx->P.eq == AF_ADVECTION || ctx->P.eq == AF_ACOUSTICS)) return coarse_step_batched(dt0);
    if (!gnx) {
      af_status s = af_ghost_fill(ctx, h, bufs, mask, 0, 0, st);
      if (s != AF_OK) return s;
    }
    return advance(0, t0, dt0, true, h->H.finest);
  }

  // Global time stepping: every level steps its interior from the same
  // synchronised state, then every coarse level takes the fine fluxes.
  af_status global_step(double t0, double dt) {
    af_status s = gnx ? AF_OK : af_ghost_fill(ctx, h, bufs, mask, 0, 0, st);
    if (s != AF_OK) return s;
    for (int l = 0; l <= h->H.finest; ++l)
      if ((s = step_level(l, t0, dt, AF_REGION_INTERIOR)) != AF_OK) return s;
    for (int l = 0; l < h->H.finest; ++l) {
      int first, count;
      af_hier_level_range(h, l, &first, &count);
      if (count && (s = af_flux_correct(ctx, h, bufs, mask, l, reg, st)) != AF_OK) return s;
    }
    return AF_OK;
  }

  af_status run(int32_t flags, double t0, double dt0) {
    // a hierarchy that is one complete level steps without a fill
    if (h->H.finest == 0) {
      int nx, ny;
      if (level_grid(h, 0, &nx, &ny) == AF_OK) {
        gnx = nx;
        gny = ny;
      }
      g_err.clear();
    }
    return (flags & AF_STEP_GLOBAL) ? global_step(t0, dt0) : coarse_step(t0, dt0);
  }
};

}  // namespace

af_status af_amr_coarse_step(af_ctx* ctx, af_hier* h, af_state* bufs, uint32_t* mask, double t0, double dt0,
                             double* flux_reg, int32_t flags, hipStream_t stream) {
  if (!ctx || !h || !mask || !flux_reg) return fail(AF_ERR_ARG, "null argument");
  af_status s = check_pair(ctx, h, bufs, "af_amr_coarse_step");
  if (s != AF_OK) return s;
  if (flags & ~(AF_STEP_GRAPH | AF_STEP_GLOBAL)) return fail(AF_ERR_ARG, "unknown flags");
  if (!std::isfinite(t0)) return fail(AF_ERR_ARG, "t0 must be finite");
  const bool global = flags & AF_STEP_GLOBAL;
  // subcycled: every level's CFL is that of level 0 (dt_l / dx_l fixed);
  // global: the finest level's
  s = check_cfl(ctx, global ? h->H.finest : 0, dt0);
  if (s != AF_OK) return s;
  if ((s = ctx_device(ctx)) != AF_OK || (s = hier_device(h)) != AF_OK) return s;
  Driver D{ctx, h, bufs, *mask, flux_reg, stream};
  if (!(flags & AF_STEP_GRAPH)) {
    s = D.run(flags, t0, dt0);
    if (s == AF_OK) *mask = D.mask;
    return s;
  }
  const GraphKey key{*mask, dt0, bufs[0].dof[0], bufs[1].dof[0], flux_reg, ctx->P.eq == AF_SWIRL ? t0 : 0.0,
                     flags};
  auto it = h->graphs.find(key);
  if (it == h->graphs.end()) {
    // a time-dependent field keys its graphs by t0 as well, so the cache is
    // bounded: when full, drain the stream and start over
    if (h->graphs.size() >= kMaxGraphs) {
      AF_HIP(hipStreamSynchronize(stream));
      for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.second);
      h->graphs.clear();
    }
    // weights and fill plans are made outside the capture
    for (int l = 0; l <= h->H.finest; ++l) {
      const double dtl = global ? dt0 : dt0 / (1 << l);
      if (ctx->P.eq == AF_ADVECTION || ctx->P.eq == AF_ACOUSTICS) weights_for(ctx, dtl / ctx->dx(l), dtl / ctx->dy(l));
      if (ctx->P.eq == AF_ACOUSTICS && !global && !weights_dev_for(ctx, dtl / ctx->dx(l), dtl / ctx->dy(l)))
        return fail(AF_ERR_DEVICE, "acoustic weight upload failed");
      if ((s = fill_plan(ctx, h, l, stream)) != AF_OK) return s;
    }
    hipStream_t cs;
    AF_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return fail(AF_ERR_DEVICE, std::string("capture: ") + hipGetErrorString(e));
    }
    Driver G{ctx, h, bufs, *mask, flux_reg, cs};
    s = G.run(flags, t0, dt0);
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (s != AF_OK) return s;
    if (e != hipSuccess) return fail(AF_ERR_DEVICE, std::string("end capture: ") + hipGetErrorString(e));
    hipGraphExec_t ex;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(AF_ERR_DEVICE, std::string("instantiate: ") + hipGetErrorString(e));
    it = h->graphs.emplace(key, ex).first;
  }
  AF_HIP(hipGraphLaunch(it->second, stream));
  // the mask after a coarse step: subcycled, level 0 flips and finer levels
  // take an even number of steps; global, every level up to the finest flips
  *mask ^= global ? ((2u << h->H.finest) - 1u) : 1u;
  return AF_OK;
}

af_status af_amr_coarse_steps(af_ctx* ctx, af_hier* h, af_state* bufs, uint32_t* mask, double t0, double dt0,
                              int32_t nsteps, double* flux_reg, int32_t flags, hipStream_t stream) {
  if (!ctx || !h || !mask || !flux_reg) return fail(AF_ERR_ARG, "null argument");
  if (nsteps <= 0) return fail(AF_ERR_ARG, "af_amr_coarse_steps: nsteps must be positive");
  if (flags & ~AF_STEP_GLOBAL) return fail(AF_ERR_ARG, "af_amr_coarse_steps: flags other than AF_STEP_GLOBAL");
  af_status s = check_pair(ctx, h, bufs, "af_amr_coarse_steps");
  if (s != AF_OK) return s;
  if (!std::isfinite(t0)) return fail(AF_ERR_ARG, "t0 must be finite");
  const bool global = flags & AF_STEP_GLOBAL;
  s = check_cfl(ctx, global ? h->H.finest : 0, dt0);
  if (s != AF_OK) return s;
  if ((s = ctx_device(ctx)) != AF_OK || (s = hier_device(h)) != AF_OK) return s;
  Driver D{ctx, h, bufs, *mask, flux_reg, stream};
  for (int32_t k = 0; k < nsteps; ++k) {
    D.defer_fix = k + 1 < nsteps;  // used by the batched path only
    s = D.run(flags, t0 + double(k) * dt0, dt0);
    if (s != AF_OK) return s;
  }
  *mask = D.mask;
  return AF_OK;
}

af_status af_amr_coarse_step_timed(af_ctx* ctx, af_hier* h, af_state* bufs, uint32_t* mask, double t0, double dt0,
                                   double* flux_reg, hipStream_t stream, void** events, int32_t max_launches,
                                   int32_t* nlaunch, double* cell_updates) {
  if (!ctx || !h || !mask || !flux_reg || !events || !nlaunch || max_launches < 0)
    return fail(AF_ERR_ARG, "null argument");
  af_status s = check_pair(ctx, h, bufs, "af_amr_coarse_step_timed");
  if (s != AF_OK) return s;
  if (!std::isfinite(t0)) return fail(AF_ERR_ARG, "t0 must be finite");
  if ((s = check_cfl(ctx, 0, dt0)) != AF_OK) return s;
  if ((s = ctx_device(ctx)) != AF_OK || (s = hier_device(h)) != AF_OK) return s;
  Driver D{ctx, h, bufs, *mask, flux_reg, stream};
  D.ev = reinterpret_cast<hipEvent_t*>(events);
  D.ev_cells = cell_updates;
  D.max_ev = max_launches;
  s = D.run(0, t0, dt0);
  *nlaunch = D.nev;
  if (s == AF_OK) *mask = D.mask;
  return s;
}

}  // extern "C"
