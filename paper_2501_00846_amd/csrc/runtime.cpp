// Host runtime of liblbm.so: argument validation, device state, tile lists,
// hipGraph replay of the step loop, autotuning, and the C ABI of include/lbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

using lbm::BoxDesc;
using lbm::Item;
using lbm::kFields;

namespace {

thread_local std::string g_create_error;

constexpr int kGraphChunk = 32;  // steps per replayed graph (even: keeps buffer parity)

struct Box {
  lbm_params prm{};
  BoxDesc desc{};
  void* mem[2] = {nullptr, nullptr};
  void* aux = nullptr;  // phi storage type; LBM_HIGH_ORDER_AC: 6 planes of n values; LBM_FINE_PHASE: 3
  void* fmem[2] = {nullptr, nullptr};  // LBM_FINE_PHASE: fine phi per parity
  int64_t n = 0;
  bool initialized = false;
  double enc_off[10] = {0};
  double enc_scale[10] = {0};
};

}  // namespace

struct lbm_ctx {
  std::vector<Box> boxes;
  int precision = 0;
  bool gc = false;  // LBM_GRADIENT_CLOSURE (all boxes)
  bool ho = false;  // LBM_HIGH_ORDER_AC (all boxes)
  bool ho_lit = false;  // with LBM_HIGH_ORDER_AC: LBM_LITERAL_ADVECTION (all boxes)
  int ho_bpb = 1;   // workgroups per box of the fourth-order flux kernel
  int ho_tiles = 1; // workgroups per box of the fourth-order phase kernel (largest box)
  bool fine = false;   // LBM_FINE_PHASE (all boxes)
  int fine_u_bpb = 1;  // with LBM_FINE_PHASE: workgroups per box of the coarse velocity kernel,
  int fine_tiles = 1;  // of the fine step kernel (tiles of the largest box)
  int fine_rbpb = 1;   // and of the restriction
  hipStream_t stream = nullptr;
  bool own_stream = false;
  lbm_device dev{};
  int parity = 0;
  lbm_tuning tuning{32, 8, 32, 0};
  bool graphs = true;
  BoxDesc* d_boxes = nullptr;
  Item* d_items = nullptr;
  int n_items = 0;
  std::vector<std::pair<int, int>> box_items;  // (first item, count) per box
  std::map<std::pair<int, int>, hipGraphExec_t> graph_cache;  // (steps, parity)
  double* d_stage = nullptr;
  int64_t stage_n = 0;
  double* d_diag = nullptr;  // diagnostics partials (n_boxes * diag_bpb values) + one result per box
  int diag_bpb = 1;          // diagnostics workgroups per box
  std::string err;
  int device = 0;
};

namespace {

lbm_status fail(lbm_ctx* c, lbm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  else g_create_error = buf;
  return s;
}

#define HIP_TRY(ctx, call)                                                                          \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess) return fail((ctx), LBM_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)


size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

void* dev_alloc(lbm_ctx* c, size_t bytes) {
  if (c->dev.alloc) return c->dev.alloc(bytes, c->dev.user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void dev_free(lbm_ctx* c, void* p) {
  if (!p) return;
  if (c->dev.free) c->dev.free(p, c->dev.user);
  else (void)hipFree(p);
}

bool finite(double v) { return std::isfinite(v); }

int nmom_of(const lbm_params& p) { return (p.flags & LBM_GRADIENT_CLOSURE) ? 4 : 10; }

lbm_status validate_box(const lbm_params& p, int idx, int precision0, const char* who = "lbm_create") {
  if (p.lattice != LBM_D3Q27) return fail(nullptr, LBM_ERR_UNSUPPORTED, "%s: box %d: lattice %d unsupported (D3Q27 only)", who, idx, p.lattice);
  if (p.nx < 1 || p.ny < 1 || p.nz < 1) return fail(nullptr, LBM_ERR_ARG, "%s: box %d: dims must be >= 1", who, idx);
  if (p.nx > (1 << 20) || p.ny > (1 << 20) || p.nz > (1 << 20)) return fail(nullptr, LBM_ERR_ARG, "%s: box %d: dims must be <= 2^20", who, idx);
  if (static_cast<int64_t>(lbm::row_pitch(LBM_BF16_OS, p.nx)) * p.ny > (int64_t(1) << 28))
    return fail(nullptr, LBM_ERR_ARG, "%s: box %d: nx (rounded up to a multiple of 32) * ny must be <= 2^28", who, idx);
  const int d[3] = {p.nx, p.ny, p.nz};
  for (int a = 0; a < 3; ++a) {
    if (p.bc[a] != LBM_PERIODIC && p.bc[a] != LBM_WALL) return fail(nullptr, LBM_ERR_ARG, "%s: box %d: bc[%d] = %d invalid", who, idx, a, p.bc[a]);
    if (p.bc[a] == LBM_WALL && d[a] < 2) return fail(nullptr, LBM_ERR_ARG, "%s: box %d: wall axis %d needs >= 2 nodes", who, idx, a);
  }
  if (p.precision < LBM_FP64 || p.precision > LBM_BF16_OS) return fail(nullptr, LBM_ERR_ARG, "%s: box %d: precision %d invalid", who, idx, p.precision);
  if (p.precision != precision0) return fail(nullptr, LBM_ERR_UNSUPPORTED, "%s: box %d: all boxes of a context must share one precision", who, idx);
  if (p.flags & ~(LBM_LITERAL_ADVECTION | LBM_GRADIENT_CLOSURE | LBM_HIGH_ORDER_AC | LBM_FINE_PHASE)) return fail(nullptr, LBM_ERR_ARG, "%s: box %d: unknown flags 0x%x", who, idx, p.flags);
  if ((p.flags & LBM_FINE_PHASE) && (p.flags & (LBM_HIGH_ORDER_AC | LBM_LITERAL_ADVECTION)))
    return fail(nullptr, LBM_ERR_UNSUPPORTED, "%s: box %d: LBM_FINE_PHASE is not combined with LBM_HIGH_ORDER_AC or LBM_LITERAL_ADVECTION", who, idx);
  // FTCS diffusion on the fine grid (spacing 1/2): stable while 4 M |l_min| <= 2,
  // l_min = -5.78 the most negative symbol of the isotropic Laplacian
  if ((p.flags & LBM_FINE_PHASE) && finite(p.mobility) && p.mobility > 2.0 / (4.0 * 5.78))
    return fail(nullptr, LBM_ERR_ARG, "%s: box %d: mobility %g too large for LBM_FINE_PHASE (stable FTCS diffusion on the fine grid needs mobility <= 0.0865)", who, idx, p.mobility);
  if (p.flags & LBM_HIGH_ORDER_AC)
    for (int a = 0; a < 3; ++a)
      if (p.bc[a] == LBM_WALL && d[a] < 4) return fail(nullptr, LBM_ERR_ARG, "%s: box %d: wall axis %d needs >= 4 nodes with LBM_HIGH_ORDER_AC", who, idx, a);
  if (!(finite(p.rho_l) && p.rho_l > 0 && finite(p.rho_g) && p.rho_g > 0)) return fail(nullptr, LBM_ERR_ARG, "%s: box %d: densities must be finite and > 0", who, idx);
  if (!(finite(p.nu_l) && p.nu_l > 0 && finite(p.nu_g) && p.nu_g > 0)) return fail(nullptr, LBM_ERR_ARG, "%s: box %d: viscosities must be finite and > 0 (tau > 1/2)", who, idx);
  if (!(finite(p.sigma) && p.sigma >= 0)) return fail(nullptr, LBM_ERR_ARG, "%s: box %d: sigma must be finite and >= 0", who, idx);
  if (!(finite(p.mobility) && p.mobility >= 0)) return fail(nullptr, LBM_ERR_ARG, "%s: box %d: mobility must be finite and >= 0", who, idx);
  if (!(finite(p.width) && p.width > 0)) return fail(nullptr, LBM_ERR_ARG, "%s: box %d: interface width must be finite and > 0", who, idx);
  if (!(finite(p.gravity[0]) && finite(p.gravity[1]) && finite(p.gravity[2]) && finite(p.rho_ref))) return fail(nullptr, LBM_ERR_ARG, "%s: box %d: gravity / rho_ref must be finite", who, idx);
  return LBM_OK;
}

void fill_desc(Box& b, int precision) { lbm::fill_box_desc(b.prm, precision, b.enc_off, b.enc_scale, b.desc); }

void default_encoding(Box& b) { lbm::default_encoding(b.enc_off, b.enc_scale); }

void drop_graphs(lbm_ctx* c) {
  for (auto& kv : c->graph_cache) (void)hipGraphExecDestroy(kv.second);
  c->graph_cache.clear();
}

lbm_status upload_boxes(lbm_ctx* c) {
  std::vector<BoxDesc> h(c->boxes.size());
  for (size_t i = 0; i < c->boxes.size(); ++i) {
    fill_desc(c->boxes[i], c->precision);
    h[i] = c->boxes[i].desc;
  }
  HIP_TRY(c, hipMemcpyAsync(c->d_boxes, h.data(), h.size() * sizeof(BoxDesc), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

// Build the tile list for the current tuning.  Items of one box are
// contiguous; within a box z-chunk is slowest, then y, then x.  The launch
// order is permuted so that workgroup b (dispatched to XCD b mod 8) gets the
// (b mod 8)-th contiguous eighth of the list: spatial neighbours, which share
// halo planes and columns, then run on the same XCD and its L2.
lbm_status build_items(lbm_ctx* c) {
  const int tx = c->tuning.block_x - 2, ty = c->tuning.block_y - 2;
  std::vector<Item> all;
  std::vector<std::pair<int, int>> box_items;
  for (size_t bi = 0; bi < c->boxes.size(); ++bi) {
    const lbm_params& p = c->boxes[bi].prm;
    const int zc = std::max(1, std::min(c->tuning.z_chunk, p.nz));
    std::vector<Item> items;
    for (int z0 = 0; z0 < p.nz; z0 += zc)
      for (int y0 = 0; y0 < p.ny; y0 += ty)
        for (int x0 = 0; x0 < p.nx; x0 += tx) {
          Item it{};
          it.box = static_cast<int>(bi);
          it.x0 = x0;
          it.y0 = y0;
          it.z0 = z0;
          it.z1 = std::min(z0 + zc, p.nz);
          items.push_back(it);
        }
    box_items.emplace_back(static_cast<int>(all.size()), static_cast<int>(items.size()));
    // XCD-contiguous permutation within the box
    const size_t n = items.size();
    const size_t per = (n + 7) / 8;
    std::vector<Item> perm;
    perm.reserve(n);
    if (c->tuning.persistent == 0 && n >= 64) {
      for (size_t b = 0; b < per * 8; ++b) {
        const size_t src = (b % 8) * per + b / 8;
        if (src < n) perm.push_back(items[src]);
      }
    } else {
      perm = items;
    }
    all.insert(all.end(), perm.begin(), perm.end());
  }
  // the new list replaces the old one only once it is on the device, so a
  // failure leaves the context on its previous, consistent tile list
  Item* d_new = static_cast<Item*>(dev_alloc(c, align256(all.size() * sizeof(Item))));
  if (!d_new) return fail(c, LBM_ERR_OOM, "tile list allocation failed");
  hipError_t e = hipMemcpyAsync(d_new, all.data(), all.size() * sizeof(Item), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    dev_free(c, d_new);
    return fail(c, LBM_ERR_DEVICE, "tile list upload failed: %s", hipGetErrorString(e));
  }
  if (c->d_items) dev_free(c, c->d_items);
  c->d_items = d_new;
  c->n_items = static_cast<int>(all.size());
  c->box_items = std::move(box_items);
  drop_graphs(c);
  return LBM_OK;
}

hipError_t enqueue_steps(lbm_ctx* c, int nsteps, int parity0) {
  int parity = parity0;
  const int grid = c->tuning.persistent > 0 ? std::min(c->tuning.persistent, c->n_items) : c->n_items;
  for (int s = 0; s < nsteps; ++s) {
    hipError_t e = lbm::launch_fused(c->precision, c->gc, c->tuning.block_x, c->tuning.block_y, c->d_boxes,
                                     c->d_items, c->n_items, grid, parity, c->stream);
    if (e != hipSuccess) return e;
    if (c->ho) {
      e = lbm::launch_high_order_phase(c->precision, c->gc, c->ho_lit, c->d_boxes, 0, static_cast<int>(c->boxes.size()),
                                       parity, c->ho_bpb, c->ho_tiles, c->stream);
      if (e != hipSuccess) return e;
    }
    if (c->fine) {
      e = lbm::launch_fine_phase(c->precision, c->gc, c->d_boxes, 0, static_cast<int>(c->boxes.size()), parity,
                                 c->fine_u_bpb, c->fine_tiles, c->fine_rbpb, c->stream);
      if (e != hipSuccess) return e;
    }
    parity ^= 1;
  }
  return hipSuccess;
}

lbm_status get_graph(lbm_ctx* c, int steps, int parity, hipGraphExec_t* out) {
  auto key = std::make_pair(steps, parity);
  auto it = c->graph_cache.find(key);
  if (it != c->graph_cache.end()) {
    *out = it->second;
    return LBM_OK;
  }
  hipGraph_t g = nullptr;
  HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
  hipError_t e = enqueue_steps(c, steps, parity);
  hipError_t e2 = hipStreamEndCapture(c->stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(c, LBM_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  }
  hipGraphExec_t ex = nullptr;
  hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e3 != hipSuccess) return fail(c, LBM_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e3));
  c->graph_cache[key] = ex;
  *out = ex;
  return LBM_OK;
}

lbm_status check_box(lbm_ctx* c, int box) {
  if (!c) return fail(nullptr, LBM_ERR_ARG, "NULL context");
  if (box < 0 || box >= static_cast<int>(c->boxes.size())) return fail(c, LBM_ERR_ARG, "box index %d out of range [0, %d)", box, static_cast<int>(c->boxes.size()));
  return LBM_OK;
}

lbm_status ensure_stage(lbm_ctx* c, int64_t n) {
  if (c->stage_n >= n) return LBM_OK;
  if (c->d_stage) dev_free(c, c->d_stage);
  c->d_stage = static_cast<double*>(dev_alloc(c, align256(static_cast<size_t>(n) * sizeof(double))));
  c->stage_n = c->d_stage ? n : 0;
  if (!c->d_stage) return fail(c, LBM_ERR_OOM, "staging buffer of %lld doubles failed", static_cast<long long>(n));
  return LBM_OK;
}

lbm_status put_field(lbm_ctx* c, Box& b, int field, const double* host) {
  if (host) HIP_TRY(c, hipMemcpyAsync(c->d_stage, host, b.n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  else HIP_TRY(c, hipMemsetAsync(c->d_stage, 0, b.n * sizeof(double), c->stream));
  HIP_TRY(c, lbm::launch_encode(c->precision, b.desc, c->parity, field, c->d_stage, b.n, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

bool all_finite(const double* v, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// lbm_diag from the kDiagValues reduced values of one box; true if the box
// holds a non-finite value.
bool fill_diag(const double* v, lbm_diag* out) {
  std::memset(out, 0, sizeof(*out));
  out->phase_mass = v[0];
  out->pstar_sum = v[1];
  for (int a = 0; a < 3; ++a) out->momentum[a] = v[2 + a];
  out->kinetic = v[5];
  out->umax = v[6];
  const double wl = v[0], wg = v[13];
  for (int a = 0; a < 3; ++a) {
    out->centroid_l[a] = wl != 0 ? v[7 + a] / wl : 0.0;
    out->velocity_l[a] = wl != 0 ? v[10 + a] / wl : 0.0;
    out->centroid_g[a] = wg != 0 ? v[14 + a] / wg : 0.0;
    out->velocity_g[a] = wg != 0 ? v[17 + a] / wg : 0.0;
  }
  out->n_l = v[21];
  out->n_g = v[23];
  out->p_l = v[21] > 0 ? v[20] / v[21] : 0.0;
  out->p_g = v[23] > 0 ? v[22] / v[23] : 0.0;
  out->nonfinite = v[24] != 0.0 || !std::isfinite(v[0]) ? 1 : 0;
  return out->nonfinite != 0;
}

// Smallest z-chunk whose tile list fits in `slots` resident workgroups, so that
// the launch runs in whole rounds of the device instead of ending on a
// partly filled one; 0 if no chunk up to maxz does.
int wave_balanced_chunk(const lbm_ctx* c, int tx, int ty, int64_t slots, int maxz) {
  for (int zc = 1; zc <= maxz; ++zc) {
    int64_t items = 0;
    for (auto& b : c->boxes) {
      const lbm_params& p = b.prm;
      const int64_t cols = static_cast<int64_t>((p.nx + tx - 1) / tx) * ((p.ny + ty - 1) / ty);
      items += cols * ((p.nz + std::min(zc, p.nz) - 1) / std::min(zc, p.nz));
    }
    if (items <= slots) return zc;
  }
  return 0;
}

}  // namespace

// Shared with the entry point that allocates nothing (noalloc.hip).
namespace lbm {

lbm_status check_params(const lbm_params& p, int idx, int precision0, const char* who) {
  return validate_box(p, idx, precision0, who);
}

lbm_status set_error(lbm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_create_error = buf;
  return s;
}

void clear_error() { g_create_error.clear(); }

int check_encoding(const double* offset, const double* scale) {
  for (int k = 0; k < 10; ++k) {
    // scale = 2^(ex-1): a power of two that FP32 holds, with its reciprocal,
    // as normal numbers, 2^-126 .. 2^126
    int ex = 0;
    const double m = std::frexp(scale[k], &ex);
    if (!(std::isfinite(scale[k]) && scale[k] > 0 && m == 0.5 && ex >= -125 && ex <= 127)) return k;
    // the kernels subtract the offset in FP32
    if (!(std::isfinite(offset[k]) && std::isfinite(static_cast<float>(offset[k])))) return 10 + k;
  }
  return -1;
}

void default_encoding(double off[10], double scale[10]) {
  // stored = (v - off) * scale: typical magnitudes land near 2^10 in FP16
  const double sP = 1024.0, sJ = 4096.0, sQ = 65536.0;
  for (int k = 0; k < 10; ++k) off[k] = 0.0;
  scale[0] = sP;
  for (int k = 1; k < 4; ++k) scale[k] = sJ;
  for (int k = 4; k < 10; ++k) scale[k] = sQ;
}

void fill_box_desc(const lbm_params& p, int precision, const double off[10], const double scale[10], BoxDesc& d) {
  d.nx = p.nx;
  d.ny = p.ny;
  d.nz = p.nz;
  for (int a = 0; a < 3; ++a) d.wall[a] = p.bc[a] == LBM_WALL ? 1 : 0;
  d.flags = p.flags;
  d.nmom = nmom_of(p);
  d.rho_g = p.rho_g;
  d.drho = p.rho_l - p.rho_g;
  d.nu_g = p.nu_g;
  d.dnu = p.nu_l - p.nu_g;
  d.beta4 = 4.0 * 12.0 * p.sigma / p.width;
  d.kappa_mu = 1.5 * p.sigma * p.width;
  d.mobility = p.mobility;
  d.kappa_ac = 4.0 * p.mobility / p.width;
  for (int a = 0; a < 3; ++a) d.grav[a] = p.gravity[a];
  d.rho_ref = p.rho_ref;
  d.pitch = row_pitch(precision, p.nx);
  bool rows = true;  // rows of pitch elements are whole 64-byte multiples
  for (int s = 0; s < 2; ++s)
    rows = rows && reinterpret_cast<uintptr_t>(d.phi[s]) % 64 == 0 && reinterpret_cast<uintptr_t>(d.mom[s]) % 64 == 0;
  d.whole_rows = rows ? 1 : 0;
  const bool os = precision == LBM_FP16_OS || precision == LBM_BF16_OS;
  d.zero_offsets = 1;
  for (int k = 0; k < 10; ++k) {
    d.enc_off[k] = os ? static_cast<float>(off[k]) : 0.f;
    d.enc_scale[k] = os ? static_cast<float>(scale[k]) : 1.f;
    d.enc_inv[k] = os ? static_cast<float>(1.0 / scale[k]) : 1.f;
    if (d.enc_off[k] != 0.f || std::signbit(d.enc_off[k])) d.zero_offsets = 0;
  }
}

}  // namespace lbm

extern "C" {

lbm_status lbm_create(const lbm_params* boxes, int32_t n_boxes, const lbm_device* dev, lbm_ctx** out) {
  try {
    g_create_error.clear();
    if (!out) return fail(nullptr, LBM_ERR_ARG, "lbm_create: out is NULL");
    *out = nullptr;
    if (!boxes) return fail(nullptr, LBM_ERR_ARG, "lbm_create: boxes is NULL");
    if (n_boxes < 1) return fail(nullptr, LBM_ERR_ARG, "lbm_create: n_boxes must be >= 1");
    for (int i = 0; i < n_boxes; ++i) {
      lbm_status s = validate_box(boxes[i], i, boxes[0].precision);
      if (s != LBM_OK) return s;
      if ((boxes[i].flags ^ boxes[0].flags) & LBM_GRADIENT_CLOSURE)
        return fail(nullptr, LBM_ERR_UNSUPPORTED, "lbm_create: box %d: all boxes of a context must share one closure", i);
      if ((boxes[i].flags ^ boxes[0].flags) & LBM_HIGH_ORDER_AC)
        return fail(nullptr, LBM_ERR_UNSUPPORTED, "lbm_create: box %d: all boxes of a context must share LBM_HIGH_ORDER_AC", i);
      if ((boxes[i].flags ^ boxes[0].flags) & LBM_FINE_PHASE)
        return fail(nullptr, LBM_ERR_UNSUPPORTED, "lbm_create: box %d: all boxes of a context must share LBM_FINE_PHASE", i);
      if ((boxes[0].flags & LBM_HIGH_ORDER_AC) && ((boxes[i].flags ^ boxes[0].flags) & LBM_LITERAL_ADVECTION))
        return fail(nullptr, LBM_ERR_UNSUPPORTED,
                    "lbm_create: box %d: with LBM_HIGH_ORDER_AC all boxes must share LBM_LITERAL_ADVECTION", i);
    }
    if (dev && ((dev->alloc == nullptr) != (dev->free == nullptr)))
      return fail(nullptr, LBM_ERR_ARG, "lbm_create: alloc and free callbacks must be given together");

    lbm_ctx* c = new lbm_ctx();
    if (dev) c->dev = *dev;
    c->precision = boxes[0].precision;
    c->gc = (boxes[0].flags & LBM_GRADIENT_CLOSURE) != 0;
    c->ho = (boxes[0].flags & LBM_HIGH_ORDER_AC) != 0;
    c->ho_lit = c->ho && (boxes[0].flags & LBM_LITERAL_ADVECTION) != 0;
    c->fine = (boxes[0].flags & LBM_FINE_PHASE) != 0;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
      delete c;
      return fail(nullptr, LBM_ERR_DEVICE, "lbm_create: no HIP device: %s", hipGetErrorString(e));
    }
    if (dev && dev->stream) {
      c->stream = static_cast<hipStream_t>(dev->stream);
    } else {
      e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
      if (e != hipSuccess) {
        delete c;
        return fail(nullptr, LBM_ERR_DEVICE, "lbm_create: stream creation failed: %s", hipGetErrorString(e));
      }
      c->own_stream = true;
    }
    c->boxes.resize(n_boxes);
    for (int i = 0; i < n_boxes; ++i) {
      Box& b = c->boxes[i];
      b.prm = boxes[i];
      b.n = static_cast<int64_t>(b.prm.nx) * b.prm.ny * b.prm.nz;
      default_encoding(b);
      // stored rows are padded to row_pitch elements (64-byte aligned rows)
      const int64_t stored = static_cast<int64_t>(lbm::row_pitch(c->precision, b.prm.nx)) * b.prm.ny * b.prm.nz;
      const size_t pb = align256(lbm::phi_bytes(c->precision, stored));
      const size_t total = pb + align256(lbm::mom_bytes(c->precision, stored, nmom_of(b.prm)));
      for (int s = 0; s < 2; ++s) {
        b.mem[s] = dev_alloc(c, total);
        if (!b.mem[s]) {
          lbm_destroy(c);
          return fail(nullptr, LBM_ERR_OOM, "lbm_create: state allocation of %zu bytes failed (box %d)", total, i);
        }
        b.desc.phi[s] = b.mem[s];
        b.desc.mom[s] = static_cast<char*>(b.mem[s]) + pb;
      }
      if (c->ho) {
        b.aux = dev_alloc(c, align256(lbm::phi_bytes(c->precision, 6 * b.n)));
        if (!b.aux) {
          lbm_destroy(c);
          return fail(nullptr, LBM_ERR_OOM, "lbm_create: high-order phase buffer allocation failed (box %d)", i);
        }
        b.desc.aux = b.aux;
      }
      if (c->fine) {
        const int64_t nf = 8 * b.n;
        b.aux = dev_alloc(c, align256(lbm::phi_bytes(c->precision, 3 * b.n)));
        for (int s = 0; s < 2; ++s) b.fmem[s] = dev_alloc(c, align256(lbm::phi_bytes(c->precision, nf)));
        if (!b.aux || !b.fmem[0] || !b.fmem[1]) {
          lbm_destroy(c);
          return fail(nullptr, LBM_ERR_OOM, "lbm_create: fine phase-field buffer allocation failed (box %d)", i);
        }
        b.desc.aux = b.aux;
        for (int s = 0; s < 2; ++s) b.desc.fphi[s] = b.fmem[s];
      }
    }
    c->d_boxes = static_cast<BoxDesc*>(dev_alloc(c, align256(n_boxes * sizeof(BoxDesc))));
    int64_t max_n = 1;
    for (auto& b : c->boxes) max_n = std::max(max_n, b.n);
    c->diag_bpb = lbm::diag_blocks_per_box(max_n);
    c->ho_bpb = lbm::high_order_blocks_per_box(max_n);
    for (auto& b : c->boxes)
      c->ho_tiles = std::max(c->ho_tiles, lbm::high_order_phase_tiles(b.prm.nx, b.prm.ny, b.prm.nz));
    if (c->fine) {
      c->fine_u_bpb = lbm::high_order_blocks_per_box(max_n);
      for (auto& b : c->boxes) {
        c->fine_tiles = std::max(c->fine_tiles, lbm::fine_tiles(b.prm.nx, b.prm.ny, b.prm.nz));
      }
      c->fine_rbpb = static_cast<int>(std::min<int64_t>(4096, (max_n + 255) / 256));
    }
    c->d_diag = static_cast<double*>(dev_alloc(
        c, align256(static_cast<size_t>(n_boxes) * (c->diag_bpb + 1) * lbm::kDiagValues * sizeof(double))));
    if (!c->d_boxes || !c->d_diag) {
      lbm_destroy(c);
      return fail(nullptr, LBM_ERR_OOM, "lbm_create: descriptor allocation failed");
    }
    // default tuning: 34 x 8 workgroups (32 x 6 output columns); z chunks
    // short enough that the tile list fills the 256 CUs several times over
    int zc = 64;
    for (; zc > 8; zc /= 2) {
      int64_t items = 0;
      for (auto& b : c->boxes)
        items += static_cast<int64_t>((b.prm.nx + 31) / 32) * ((b.prm.ny + 5) / 6) * ((b.prm.nz + zc - 1) / zc);
      if (items >= 2048) break;
    }
    c->tuning = lbm_tuning{34, 8, zc, 0};
    lbm_status s = upload_boxes(c);
    if (s == LBM_OK) s = build_items(c);
    if (s != LBM_OK) {
      g_create_error = c->err;
      lbm_destroy(c);
      return s;
    }
    *out = c;
    return LBM_OK;
  } catch (const std::bad_alloc&) {
    return fail(nullptr, LBM_ERR_OOM, "lbm_create: host allocation failed");
  } catch (...) {
    return fail(nullptr, LBM_ERR_DEVICE, "lbm_create: unexpected exception");
  }
}

lbm_status lbm_init_phase(lbm_ctx* c, int32_t box, const double* phi, const double* u, const double* pstar) {
  lbm_status s = check_box(c, box);
  if (s != LBM_OK) return s;
  if (!phi) return fail(c, LBM_ERR_ARG, "lbm_init_phase: phi is NULL");
  Box& b = c->boxes[box];
  s = ensure_stage(c, b.n);
  if (s != LBM_OK) return s;
  if ((s = put_field(c, b, 0, phi)) != LBM_OK) return s;
  if ((s = put_field(c, b, 1, pstar)) != LBM_OK) return s;
  for (int a = 0; a < 3; ++a)
    if ((s = put_field(c, b, 2 + a, u ? u + a * b.n : nullptr)) != LBM_OK) return s;
  for (int k = 5; k < kFields; ++k)
    if ((s = put_field(c, b, k, nullptr)) != LBM_OK) return s;
  if (c->fine) {
    HIP_TRY(c, lbm::launch_fine_init(c->precision, b.desc, c->d_boxes + box, c->parity, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  b.initialized = true;
  return LBM_OK;
}

lbm_status lbm_set_state(lbm_ctx* c, int32_t box, const double* state) {
  lbm_status s = check_box(c, box);
  if (s != LBM_OK) return s;
  if (!state) return fail(c, LBM_ERR_ARG, "lbm_set_state: state is NULL");
  Box& b = c->boxes[box];
  if ((s = ensure_stage(c, b.n)) != LBM_OK) return s;
  for (int k = 0; k < kFields; ++k)
    if ((s = put_field(c, b, k, state + k * b.n)) != LBM_OK) return s;
  if (c->fine) {
    HIP_TRY(c, lbm::launch_fine_init(c->precision, b.desc, c->d_boxes + box, c->parity, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  b.initialized = true;
  return LBM_OK;
}

lbm_status lbm_get_fine_phase(lbm_ctx* c, int32_t box, double* out) {
  lbm_status s = check_box(c, box);
  if (s != LBM_OK) return s;
  if (!out) return fail(c, LBM_ERR_ARG, "lbm_get_fine_phase: out is NULL");
  if (!c->fine) return fail(c, LBM_ERR_UNSUPPORTED, "lbm_get_fine_phase: the context has no LBM_FINE_PHASE");
  Box& b = c->boxes[box];
  if (!b.initialized) return fail(c, LBM_ERR_STATE, "lbm_get_fine_phase: box %d not initialised", box);
  const int64_t nf = 8 * b.n;
  if ((s = ensure_stage(c, nf)) != LBM_OK) return s;
  HIP_TRY(c, lbm::launch_fine_get(c->precision, b.desc, c->parity, c->d_stage, c->stream));
  HIP_TRY(c, hipMemcpyAsync(out, c->d_stage, nf * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (!all_finite(out, nf)) return fail(c, LBM_ERR_UNSTABLE, "lbm_get_fine_phase: non-finite values in box %d", box);
  return LBM_OK;
}

lbm_status lbm_get_fine_phase_points(lbm_ctx* c, int32_t box, int64_t n, const int64_t* node, double* out) {
  lbm_status s = check_box(c, box);
  if (s != LBM_OK) return s;
  if (n < 0 || (n > 0 && (!node || !out)))
    return fail(c, LBM_ERR_ARG, "lbm_get_fine_phase_points: bad n / NULL arrays");
  if (!c->fine) return fail(c, LBM_ERR_UNSUPPORTED, "lbm_get_fine_phase_points: the context has no LBM_FINE_PHASE");
  Box& b = c->boxes[box];
  if (!b.initialized) return fail(c, LBM_ERR_STATE, "lbm_get_fine_phase_points: box %d not initialised", box);
  for (int64_t j = 0; j < n; ++j)
    if (node[j] < 0 || node[j] >= 8 * b.n)
      return fail(c, LBM_ERR_ARG, "lbm_get_fine_phase_points: node[%lld] out of range", static_cast<long long>(j));
  if (n == 0) return LBM_OK;
  // staging: n indices (as doubles' storage) + n values
  if ((s = ensure_stage(c, 2 * n)) != LBM_OK) return s;
  int64_t* d_idx = reinterpret_cast<int64_t*>(c->d_stage);
  double* d_out = c->d_stage + n;
  HIP_TRY(c, hipMemcpyAsync(d_idx, node, n * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, lbm::launch_fine_gather(c->precision, b.desc, c->parity, d_idx, n, d_out, c->stream));
  HIP_TRY(c, hipMemcpyAsync(out, d_out, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_set_fine_phase(lbm_ctx* c, int32_t box, const double* in) {
  lbm_status s = check_box(c, box);
  if (s != LBM_OK) return s;
  if (!in) return fail(c, LBM_ERR_ARG, "lbm_set_fine_phase: in is NULL");
  if (!c->fine) return fail(c, LBM_ERR_UNSUPPORTED, "lbm_set_fine_phase: the context has no LBM_FINE_PHASE");
  Box& b = c->boxes[box];
  if (!b.initialized) return fail(c, LBM_ERR_STATE, "lbm_set_fine_phase: box %d holds no state", box);
  const int64_t nf = 8 * b.n;
  if ((s = ensure_stage(c, nf)) != LBM_OK) return s;
  HIP_TRY(c, hipMemcpyAsync(c->d_stage, in, nf * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, lbm::launch_fine_set(c->precision, b.desc, c->d_boxes + box, c->parity, c->d_stage, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_get_state(lbm_ctx* c, int32_t box, double* state) {
  lbm_status s = check_box(c, box);
  if (s != LBM_OK) return s;
  if (!state) return fail(c, LBM_ERR_ARG, "lbm_get_state: state is NULL");
  Box& b = c->boxes[box];
  if (!b.initialized) return fail(c, LBM_ERR_STATE, "lbm_get_state: box %d not initialised", box);
  if ((s = ensure_stage(c, b.n)) != LBM_OK) return s;
  for (int k = 0; k < kFields; ++k) {
    HIP_TRY(c, lbm::launch_decode(c->precision, b.desc, c->parity, k, c->d_stage, b.n, c->stream));
    HIP_TRY(c, hipMemcpyAsync(state + k * b.n, c->d_stage, b.n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  if (!all_finite(state, kFields * b.n)) return fail(c, LBM_ERR_UNSTABLE, "lbm_get_state: non-finite state");
  return LBM_OK;
}

lbm_status lbm_get_state_points(lbm_ctx* c, int32_t box, int64_t n, const int64_t* node, double* out) {
  lbm_status s = check_box(c, box);
  if (s != LBM_OK) return s;
  if (n < 0 || (n > 0 && (!node || !out))) return fail(c, LBM_ERR_ARG, "lbm_get_state_points: bad n / NULL arrays");
  Box& b = c->boxes[box];
  if (!b.initialized) return fail(c, LBM_ERR_STATE, "lbm_get_state_points: box %d not initialised", box);
  for (int64_t j = 0; j < n; ++j)
    if (node[j] < 0 || node[j] >= b.n) return fail(c, LBM_ERR_ARG, "lbm_get_state_points: node[%lld] out of range", static_cast<long long>(j));
  if (n == 0) return LBM_OK;
  // staging: n indices (as doubles' storage) + 11 n values
  if ((s = ensure_stage(c, 12 * n)) != LBM_OK) return s;
  int64_t* d_idx = reinterpret_cast<int64_t*>(c->d_stage);
  double* d_out = c->d_stage + n;
  HIP_TRY(c, hipMemcpyAsync(d_idx, node, n * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, lbm::launch_gather(c->precision, b.desc, c->parity, d_idx, n, d_out, c->stream));
  HIP_TRY(c, hipMemcpyAsync(out, d_out, 11 * n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int32_t nsteps) {
  if (!c) return fail(nullptr, LBM_ERR_ARG, "NULL context");
  if (nsteps < 0) return fail(c, LBM_ERR_ARG, "lbm_step: nsteps must be >= 0");
  for (size_t i = 0; i < c->boxes.size(); ++i)
    if (!c->boxes[i].initialized) return fail(c, LBM_ERR_STATE, "lbm_step: box %zu not initialised", i);
  if (nsteps == 0) return LBM_OK;
  if (!c->graphs) {
    HIP_TRY(c, enqueue_steps(c, nsteps, c->parity));
    c->parity ^= (nsteps & 1);
    return LBM_OK;
  }
  int left = nsteps;
  while (left > 0) {
    const int k = left >= kGraphChunk ? kGraphChunk : left;
    hipGraphExec_t ex = nullptr;
    lbm_status s = get_graph(c, k, c->parity, &ex);
    if (s != LBM_OK) return s;
    HIP_TRY(c, hipGraphLaunch(ex, c->stream));
    c->parity ^= (k & 1);
    left -= k;
  }
  return LBM_OK;
}

lbm_status lbm_step_unbatched(lbm_ctx* c, int32_t nsteps) {
  if (!c) return fail(nullptr, LBM_ERR_ARG, "NULL context");
  if (nsteps < 0) return fail(c, LBM_ERR_ARG, "lbm_step_unbatched: nsteps must be >= 0");
  for (size_t i = 0; i < c->boxes.size(); ++i)
    if (!c->boxes[i].initialized) return fail(c, LBM_ERR_STATE, "lbm_step_unbatched: box %zu not initialised", i);
  for (int s = 0; s < nsteps; ++s) {
    for (size_t k = 0; k < c->box_items.size(); ++k) {
      const auto& bi = c->box_items[k];
      HIP_TRY(c, lbm::launch_fused(c->precision, c->gc, c->tuning.block_x, c->tuning.block_y, c->d_boxes,
                                   c->d_items + bi.first, bi.second, bi.second, c->parity, c->stream));
      if (c->ho)
        HIP_TRY(c, lbm::launch_high_order_phase(c->precision, c->gc, c->ho_lit, c->d_boxes, static_cast<int>(k), 1,
                                                c->parity, c->ho_bpb, c->ho_tiles, c->stream));
      if (c->fine)
        HIP_TRY(c, lbm::launch_fine_phase(c->precision, c->gc, c->d_boxes, static_cast<int>(k), 1, c->parity,
                                          c->fine_u_bpb, c->fine_tiles, c->fine_rbpb, c->stream));
    }
    c->parity ^= 1;
  }
  return LBM_OK;
}

lbm_status lbm_get_fields(lbm_ctx* c, int32_t box, double* rho, double* u, double* phi, double* p) {
  lbm_status s = check_box(c, box);
  if (s != LBM_OK) return s;
  Box& b = c->boxes[box];
  if (!b.initialized) return fail(c, LBM_ERR_STATE, "lbm_get_fields: box %d not initialised", box);
  if ((s = ensure_stage(c, b.n)) != LBM_OK) return s;
  double* outs[6] = {rho, u, u ? u + b.n : nullptr, u ? u + 2 * b.n : nullptr, phi, p};
  bool fin = true;
  for (int w = 0; w < 6; ++w) {
    if (!outs[w]) continue;
    HIP_TRY(c, lbm::launch_observable(c->precision, b.desc, c->parity, w, c->d_stage, c->stream));
    HIP_TRY(c, hipMemcpyAsync(outs[w], c->d_stage, b.n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    fin = fin && all_finite(outs[w], b.n);
  }
  if (!fin) return fail(c, LBM_ERR_UNSTABLE, "lbm_get_fields: non-finite values in box %d", box);
  return LBM_OK;
}

lbm_status lbm_diagnostics(lbm_ctx* c, int32_t box, lbm_diag* out) {
  lbm_status s = check_box(c, box);
  if (s != LBM_OK) return s;
  if (!out) return fail(c, LBM_ERR_ARG, "lbm_diagnostics: out is NULL");
  Box& b = c->boxes[box];
  if (!b.initialized) return fail(c, LBM_ERR_STATE, "lbm_diagnostics: box %d not initialised", box);
  double* d_out = c->d_diag + static_cast<size_t>(c->boxes.size()) * c->diag_bpb * lbm::kDiagValues;
  HIP_TRY(c, lbm::launch_diagnostics(c->precision, c->gc, c->d_boxes, box, 1, c->parity, c->diag_bpb, c->d_diag, d_out,
                                     c->stream));
  double v[lbm::kDiagValues];
  HIP_TRY(c, hipMemcpyAsync(v, d_out, sizeof(v), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (fill_diag(v, out)) return fail(c, LBM_ERR_UNSTABLE, "lbm_diagnostics: non-finite state in box %d", box);
  return LBM_OK;
}

lbm_status lbm_diagnostics_all(lbm_ctx* c, lbm_diag* out) {
  if (!c) return fail(nullptr, LBM_ERR_ARG, "NULL context");
  if (!out) return fail(c, LBM_ERR_ARG, "lbm_diagnostics_all: out is NULL");
  const int nb = static_cast<int>(c->boxes.size());
  for (int i = 0; i < nb; ++i)
    if (!c->boxes[i].initialized) return fail(c, LBM_ERR_STATE, "lbm_diagnostics_all: box %d not initialised", i);
  double* d_out = c->d_diag + static_cast<size_t>(nb) * c->diag_bpb * lbm::kDiagValues;
  HIP_TRY(c, lbm::launch_diagnostics(c->precision, c->gc, c->d_boxes, 0, nb, c->parity, c->diag_bpb, c->d_diag, d_out,
                                     c->stream));
  std::vector<double> v(static_cast<size_t>(nb) * lbm::kDiagValues);
  HIP_TRY(c, hipMemcpyAsync(v.data(), d_out, v.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int bad = -1;
  for (int i = 0; i < nb; ++i)
    if (fill_diag(v.data() + static_cast<size_t>(i) * lbm::kDiagValues, out + i) && bad < 0) bad = i;
  if (bad >= 0) return fail(c, LBM_ERR_UNSTABLE, "lbm_diagnostics_all: non-finite state in box %d", bad);
  return LBM_OK;
}

lbm_status lbm_set_encoding(lbm_ctx* c, int32_t box, const double* offset, const double* scale) {
  lbm_status s = check_box(c, box);
  if (s != LBM_OK) return s;
  if (!offset || !scale) return fail(c, LBM_ERR_ARG, "lbm_set_encoding: NULL offset/scale");
  const int bad = lbm::check_encoding(offset, scale);
  if (bad >= 10) return fail(c, LBM_ERR_ARG, "lbm_set_encoding: offset[%d] must be finite in FP32", bad - 10);
  if (bad >= 0) return fail(c, LBM_ERR_ARG, "lbm_set_encoding: scale[%d] must be a power of two in [2^-126, 2^126]", bad);
  Box& b = c->boxes[box];
  if (c->precision != LBM_FP16_OS && c->precision != LBM_BF16_OS) return LBM_OK;
  const BoxDesc before = b.desc;
  double keep_off[10], keep_scale[10];
  for (int k = 0; k < 10; ++k) {
    keep_off[k] = b.enc_off[k];
    keep_scale[k] = b.enc_scale[k];
    b.enc_off[k] = offset[k];
    b.enc_scale[k] = scale[k];
  }
  fill_desc(b, c->precision);
  if (b.initialized) {
    // re-encode the live moments: decode each field with the previous
    // encoding into the staging buffer, encode it again with the new one
    lbm_status st = ensure_stage(c, b.n);
    for (int k = 0; st == LBM_OK && k < b.desc.nmom; ++k) {
      hipError_t e = lbm::launch_decode(c->precision, before, c->parity, 1 + k, c->d_stage, b.n, c->stream);
      if (e == hipSuccess) e = lbm::launch_encode(c->precision, b.desc, c->parity, 1 + k, c->d_stage, b.n, c->stream);
      if (e != hipSuccess) st = fail(c, LBM_ERR_DEVICE, "lbm_set_encoding: re-encoding failed: %s", hipGetErrorString(e));
    }
    if (st != LBM_OK) {
      // the state may be partly re-encoded: it no longer matches either encoding
      for (int k = 0; k < 10; ++k) {
        b.enc_off[k] = keep_off[k];
        b.enc_scale[k] = keep_scale[k];
      }
      b.initialized = false;
      (void)upload_boxes(c);
      return st;
    }
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return upload_boxes(c);
}

lbm_status lbm_set_tuning(lbm_ctx* c, const lbm_tuning* t) {
  if (!c) return fail(nullptr, LBM_ERR_ARG, "NULL context");
  if (!t) return fail(c, LBM_ERR_ARG, "lbm_set_tuning: NULL tuning");
  if (!lbm::fused_config_supported(c->precision, c->gc, t->block_x, t->block_y)) return fail(c, LBM_ERR_UNSUPPORTED, "lbm_set_tuning: block %dx%d unsupported for this precision and closure", t->block_x, t->block_y);
  if (t->z_chunk < 1) return fail(c, LBM_ERR_ARG, "lbm_set_tuning: z_chunk must be >= 1");
  if (t->persistent < 0) return fail(c, LBM_ERR_ARG, "lbm_set_tuning: persistent must be >= 0");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const lbm_tuning before = c->tuning;
  c->tuning = *t;
  lbm_status s = build_items(c);
  if (s != LBM_OK) c->tuning = before;  // the previous tile list is still in place
  return s;
}

lbm_status lbm_get_tuning(const lbm_ctx* c, lbm_tuning* t) {
  if (!c || !t) return fail(const_cast<lbm_ctx*>(c), LBM_ERR_ARG, "lbm_get_tuning: NULL argument");
  *t = c->tuning;
  return LBM_OK;
}

lbm_status lbm_set_graphs(lbm_ctx* c, int32_t enabled) {
  if (!c) return fail(nullptr, LBM_ERR_ARG, "NULL context");
  c->graphs = enabled != 0;
  return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx* c, int32_t steps, lbm_tuning* best) {
  if (!c) return fail(nullptr, LBM_ERR_ARG, "NULL context");
  if (steps < 1) return fail(c, LBM_ERR_ARG, "lbm_autotune: steps must be >= 1");
  for (size_t i = 0; i < c->boxes.size(); ++i)
    if (!c->boxes[i].initialized) return fail(c, LBM_ERR_STATE, "lbm_autotune: box %zu not initialised", i);
  const int shapes[5][2] = {{32, 8}, {34, 8}, {34, 15}, {18, 14}, {66, 8}};
  int maxz = 1;
  for (auto& b : c->boxes) maxz = std::max(maxz, b.prm.nz);
  std::vector<int> fixed_zcs;
  for (int z : {2, 4, 8, 16, 32, 64, 128})
    if (z <= maxz) fixed_zcs.push_back(z);
  if (fixed_zcs.empty() || fixed_zcs.back() < maxz) fixed_zcs.push_back(maxz);
  int dev = 0, cus = 0;
  HIP_TRY(c, hipGetDevice(&dev));
  HIP_TRY(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  const bool graphs = c->graphs;
  c->graphs = true;
  struct Cand {
    lbm_tuning t;
    float ms;
  };
  std::vector<Cand> cands;
  for (auto& sh : shapes) {
    if (!lbm::fused_config_supported(c->precision, c->gc, sh[0], sh[1])) continue;
    std::vector<int> zcs = fixed_zcs;
    const int slots = cus * lbm::fused_blocks_per_cu(c->precision, c->gc, sh[0], sh[1]);
    for (int rounds = 1; slots > 0 && rounds <= 4; ++rounds) {
      const int zc = wave_balanced_chunk(c, sh[0] - 2, sh[1] - 2, static_cast<int64_t>(rounds) * slots, maxz);
      if (zc >= 2 && std::find(zcs.begin(), zcs.end(), zc) == zcs.end()) zcs.push_back(zc);
    }
    for (int zc : zcs) cands.push_back({lbm_tuning{sh[0], sh[1], zc, 0}, 1e30f});
  }
  // time `n` steps of candidate k; each candidate keeps its fastest time
  auto time_cand = [&](Cand& k, int n) -> lbm_status {
    lbm_status s = lbm_set_tuning(c, &k.t);
    if (s != LBM_OK) return s;
    if ((s = lbm_step(c, 2)) != LBM_OK) return s;
    HIP_TRY(c, hipEventRecord(e0, c->stream));
    if ((s = lbm_step(c, n)) != LBM_OK) return s;
    HIP_TRY(c, hipEventRecord(e1, c->stream));
    HIP_TRY(c, hipEventSynchronize(e1));
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
    k.ms = std::min(k.ms, ms / static_cast<float>(n));
    return LBM_OK;
  };
  // one pass over every candidate, then two more passes (in opposite orders)
  // over the finalists within 5 % of the best, so that the choice between
  // near-equal launches rests on the best of three timings rather than on
  // one noisy sample
  auto search = [&]() -> lbm_status {
    for (auto& k : cands)
      if (lbm_status s = time_cand(k, steps); s != LBM_OK) return s;
    float first = 1e30f;
    for (auto& k : cands) first = std::min(first, k.ms);
    std::vector<size_t> fin;
    for (size_t i = 0; i < cands.size(); ++i)
      if (cands[i].ms <= 1.05f * first) fin.push_back(i);
    // re-timings span at least ~25 ms each, so that small boxes are not
    // decided on a few hundred microseconds of launches
    const int n2 = std::min(4096, std::max(2 * steps, static_cast<int>(25.0f / std::max(first, 1e-4f)) + 1));
    for (int pass = 0; pass < 2 && fin.size() > 1; ++pass)
      for (size_t j = 0; j < fin.size(); ++j) {
        Cand& k = cands[fin[pass == 0 ? j : fin.size() - 1 - j]];
        if (lbm_status s = time_cand(k, n2); s != LBM_OK) return s;
      }
    return LBM_OK;
  };
  const lbm_tuning before = c->tuning;
  lbm_status s = search();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->graphs = graphs;
  lbm_tuning best_t = before;
  float best_ms = 1e30f;
  for (auto& k : cands)
    if (k.ms < best_ms) {
      best_ms = k.ms;
      best_t = k.t;
    }
  if (s != LBM_OK) {
    // leave the context on the launch it had; the error message is kept
    (void)lbm_set_tuning(c, &before);
    return s;
  }
  if ((s = lbm_set_tuning(c, &best_t)) != LBM_OK) return s;
  if (best) *best = best_t;
  return LBM_OK;
}

lbm_status lbm_synchronize(lbm_ctx* c) {
  if (!c) return fail(nullptr, LBM_ERR_ARG, "NULL context");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

double lbm_bytes_per_update(const lbm_ctx* c) {
  if (!c) return 0.0;
  return 2.0 * static_cast<double>(lbm::phi_bytes(c->precision, 1) + lbm::mom_bytes(c->precision, 1, c->gc ? 4 : 10));
}

int64_t lbm_total_nodes(const lbm_ctx* c) {
  if (!c) return 0;
  int64_t n = 0;
  for (auto& b : c->boxes) n += b.n;
  return n;
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  for (auto& b : c->boxes) {
    for (int s = 0; s < 2; ++s) dev_free(c, b.mem[s]);
    for (int s = 0; s < 2; ++s) dev_free(c, b.fmem[s]);
    dev_free(c, b.aux);
  }
  dev_free(c, c->d_boxes);
  dev_free(c, c->d_items);
  dev_free(c, c->d_stage);
  dev_free(c, c->d_diag);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* lbm_last_error(const lbm_ctx* c) {
  if (!c) return g_create_error.c_str();
  return c->err.c_str();
}

}  // extern "C"
