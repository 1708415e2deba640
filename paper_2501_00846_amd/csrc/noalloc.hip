// lbm_step_noalloc: the fused step of one box whose state lives in device
// buffers the caller owns, for callers that cannot allocate device memory
// (code under stream capture, tight serving loops).  The only device memory
// the step needs beyond that state -- the box descriptor and the tile list
// that the fused kernel reads -- lives in `scratch`, a fixed array of this
// file with static storage on every GPU the library runs on.  The call
// allocates nothing: no hipMalloc, no hipFree, no allocating library routine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "lbm.h"
#include "lbm_internal.h"

namespace lbm {
namespace {

// Layout of scratch: the descriptor of the box (first kDescBytes), then the
// tile list.  1 MiB holds 32,736 items: a 512^3 box with 32 x 13 output
// columns per tile needs 640 tiles per z-chunk, so any z-chunk >= 11 fits.
constexpr size_t kScratchBytes = size_t(1) << 20;
constexpr size_t kDescBytes = 1024;
constexpr int64_t kMaxItems = static_cast<int64_t>((kScratchBytes - kDescBytes) / sizeof(Item));
static_assert(sizeof(BoxDesc) <= kDescBytes, "descriptor slot too small");
static_assert(kDescBytes % alignof(Item) == 0, "tile list misaligned");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of scratch per device (hipGetSymbolAddress once per device,
// with that device current).  The host-side name `scratch` is only a handle
// for the runtime and is never passed to a kernel or a copy.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {};

hipError_t scratch_address(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

// Writes the descriptor and the tile list into buf (the device address of
// scratch).  The tiles of the box in natural order (z-chunk slowest, then y,
// then x) are permuted as the context API orders them: launch position b of
// per*8 slots takes natural tile (b mod 8)*per + b/8 when that index exists,
// and the slots without a tile are squeezed out, so that each eighth of the
// list -- the workgroups one XCD receives -- covers one contiguous block of
// tiles.  Thread b handles slot b.
__global__ void noalloc_setup(unsigned char* __restrict__ buf, BoxDesc desc, int tx, int ty, int zc,
                              int ntx, int nty, int n, int per, int permute) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0) *reinterpret_cast<BoxDesc*>(buf) = desc;
  Item* items = reinterpret_cast<Item*>(buf + kDescBytes);
  int src = b, pos = b;
  if (permute) {
    if (b >= per * 8) return;
    src = (b % 8) * per + b / 8;
    if (src >= n) return;
    // slots before b whose natural index falls beyond the list: residue r,
    // quotient q with 8 q + r < b and r * per + q >= n
    int empty = 0;
    for (int r = 0; r < 8; ++r) {
      const int qhi = b > r ? (b - r + 7) / 8 : 0;
      const int qlo = std::max(0, n - r * per);
      empty += std::max(0, qhi - qlo);
    }
    pos = b - empty;
  } else if (b >= n) {
    return;
  }
  const int xi = src % ntx, yi = (src / ntx) % nty, zi = src / (ntx * nty);
  Item it{};
  it.box = 0;
  it.x0 = xi * tx;
  it.y0 = yi * ty;
  it.z0 = zi * zc;
  it.z1 = std::min(it.z0 + zc, desc.nz);
  items[pos] = it;
}

}  // namespace
}  // namespace lbm

extern "C" lbm_status lbm_step_noalloc(const lbm_params* box, const lbm_tuning* tuning, void* const phi[2],
                                       void* const mom[2], const double* enc_offset, const double* enc_scale,
                                       int32_t parity, int32_t nsteps, void* stream) {
  using namespace lbm;
  const char* who = "lbm_step_noalloc";
  clear_error();
  if (!box) return set_error(LBM_ERR_ARG, "%s: box is NULL", who);
  lbm_status s = check_params(*box, 0, box->precision, who);
  if (s != LBM_OK) return s;
  if (box->flags & LBM_HIGH_ORDER_AC)
    return set_error(LBM_ERR_UNSUPPORTED, "%s: LBM_HIGH_ORDER_AC needs per-box device buffers; use a context", who);
  if (box->flags & LBM_FINE_PHASE)
    return set_error(LBM_ERR_UNSUPPORTED, "%s: LBM_FINE_PHASE needs per-box device buffers; use a context", who);
  if (!phi || !mom) return set_error(LBM_ERR_ARG, "%s: phi / mom buffer arrays are NULL", who);
  const int prec = box->precision;
  const size_t ep = prec == LBM_FP64 ? 8 : 4;
  const size_t em = prec == LBM_FP64 ? 8 : (prec == LBM_FP32 ? 4 : 2);
  for (int k = 0; k < 2; ++k) {
    if (!phi[k] || !mom[k]) return set_error(LBM_ERR_ARG, "%s: state buffer %d is NULL", who, k);
    if (reinterpret_cast<uintptr_t>(phi[k]) % ep != 0 || reinterpret_cast<uintptr_t>(mom[k]) % em != 0)
      return set_error(LBM_ERR_ARG, "%s: state buffer %d is not aligned to its element size", who, k);
  }
  if (parity != 0 && parity != 1) return set_error(LBM_ERR_ARG, "%s: parity must be 0 or 1", who);
  if (nsteps < 0) return set_error(LBM_ERR_ARG, "%s: nsteps must be >= 0", who);
  if ((enc_offset == nullptr) != (enc_scale == nullptr))
    return set_error(LBM_ERR_ARG, "%s: enc_offset and enc_scale must be given together", who);
  double off[10], scale[10];
  default_encoding(off, scale);
  if (enc_offset) {
    const int bad = check_encoding(enc_offset, enc_scale);
    if (bad >= 10) return set_error(LBM_ERR_ARG, "%s: enc_offset[%d] must be finite in FP32", who, bad - 10);
    if (bad >= 0) return set_error(LBM_ERR_ARG, "%s: enc_scale[%d] must be a power of two in [2^-126, 2^126]", who, bad);
    std::copy(enc_offset, enc_offset + 10, off);
    std::copy(enc_scale, enc_scale + 10, scale);
  }
  const bool gc = (box->flags & LBM_GRADIENT_CLOSURE) != 0;
  lbm_tuning t{34, 15, 0, 0};
  if (tuning) {
    t = *tuning;
    if (!fused_config_supported(prec, gc, t.block_x, t.block_y))
      return set_error(LBM_ERR_UNSUPPORTED, "%s: block %dx%d unsupported for this precision and closure", who,
                       t.block_x, t.block_y);
    if (t.z_chunk < 1) return set_error(LBM_ERR_ARG, "%s: z_chunk must be >= 1", who);
    if (t.persistent < 0) return set_error(LBM_ERR_ARG, "%s: persistent must be >= 0", who);
  }
  const int tx = t.block_x - 2, ty = t.block_y - 2;
  const int64_t ntx = (box->nx + tx - 1) / tx, nty = (box->ny + ty - 1) / ty;
  auto items_for = [&](int zc) { return ntx * nty * ((box->nz + zc - 1) / zc); };
  if (!tuning) {
    // z-chunks short enough to fill the 256 CUs several times over, long
    // enough for the tile list to fit the scratch array
    int zc = std::min(64, box->nz);
    while (zc > 8 && items_for(zc) < 2048) zc /= 2;
    while (items_for(zc) > kMaxItems && zc < box->nz) zc = std::min(box->nz, 2 * zc);
    t.z_chunk = zc;
  }
  const int zc = std::min(t.z_chunk, box->nz);
  const int64_t n = items_for(zc);
  if (n > kMaxItems)
    return set_error(LBM_ERR_ARG, "%s: %lld tiles exceed the %lld the static scratch array holds; use a larger z_chunk",
                     who, static_cast<long long>(n), static_cast<long long>(kMaxItems));
  if (nsteps == 0) return LBM_OK;

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(LBM_ERR_DEVICE, "%s: no HIP device: %s", who, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(LBM_ERR_UNSUPPORTED, "%s: device %d beyond %d", who, dev, kMaxDevices);
  unsigned char* buf = nullptr;
  e = scratch_address(dev, &buf);
  if (e != hipSuccess) return set_error(LBM_ERR_DEVICE, "%s: hipGetSymbolAddress failed: %s", who, hipGetErrorString(e));

  BoxDesc d{};
  for (int k = 0; k < 2; ++k) {
    d.phi[k] = phi[k];
    d.mom[k] = mom[k];
  }
  fill_box_desc(*box, prec, off, scale, d);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const int ni = static_cast<int>(n);
  const int per = (ni + 7) / 8;
  const int permute = (t.persistent == 0 && ni >= 64) ? 1 : 0;
  const int slots = permute ? per * 8 : ni;
  hipLaunchKernelGGL(noalloc_setup, dim3((slots + 255) / 256), dim3(256), 0, st, buf, d, tx, ty, zc,
                     static_cast<int>(ntx), static_cast<int>(nty), ni, per, permute);
  e = hipGetLastError();
  if (e != hipSuccess) return set_error(LBM_ERR_DEVICE, "%s: setup launch failed: %s", who, hipGetErrorString(e));
  const BoxDesc* d_desc = reinterpret_cast<const BoxDesc*>(buf);
  const Item* d_items = reinterpret_cast<const Item*>(buf + kDescBytes);
  const int grid = t.persistent > 0 ? std::min(t.persistent, ni) : ni;
  int p = parity;
  for (int k = 0; k < nsteps; ++k) {
    e = launch_fused(prec, gc, t.block_x, t.block_y, d_desc, d_items, ni, grid, p, st);
    if (e != hipSuccess) return set_error(LBM_ERR_DEVICE, "%s: step launch failed: %s", who, hipGetErrorString(e));
    p ^= 1;
  }
  return LBM_OK;
}
