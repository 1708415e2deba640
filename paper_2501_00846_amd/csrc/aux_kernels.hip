// Device code of liblbm.so beyond the fused step: encoding of host fields
// into the storage formats and back, sampled readback, the observables
// (rho, u, phi, p), the FP64 diagnostics reductions, and the two kernels of
// the fourth-order phase-field variant.  None of them runs in the step loop
// except the fourth-order kernels, and those only with LBM_HIGH_ORDER_AC.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device_common.h"
#include "lbm_internal.h"

namespace lbm {
namespace {

// ---------------------------------------------------------------------------
// Non-hot kernels: encode / decode / observables / diagnostics
// ---------------------------------------------------------------------------
// Storage offsets: rows are b.pitch elements apart.  Node (x, y, z) of phi,
// and moment k of that node.
__device__ __forceinline__ int64_t phi_at(const BoxDesc& b, int x, int y, int z) {
  return (static_cast<int64_t>(z) * b.ny + y) * b.pitch + x;
}
__device__ __forceinline__ int64_t mom_at(const BoxDesc& b, int k, int x, int y, int z) {
  return ((static_cast<int64_t>(z) * b.nmom + k) * b.ny + y) * b.pitch + x;
}
// coordinates of the flat node index i = x + nx (y + ny z)
// (32-bit divisions whenever the index fits, which covers boxes of up to
// 2^32 nodes; 64-bit ones beyond)
__device__ __forceinline__ void node_xyz(const BoxDesc& b, int64_t i, int& x, int& y, int& z) {
  if (static_cast<uint64_t>(i) <= 0xffffffffull) {
    const uint32_t ii = static_cast<uint32_t>(i), unx = static_cast<uint32_t>(b.nx), uny = static_cast<uint32_t>(b.ny);
    const uint32_t r = ii / unx;
    x = static_cast<int>(ii - r * unx);
    y = static_cast<int>(r % uny);
    z = static_cast<int>(r / uny);
    return;
  }
  const int64_t r = i / b.nx;
  x = static_cast<int>(i - r * b.nx);
  y = static_cast<int>(r % b.ny);
  z = static_cast<int>(r / b.ny);
}

template <class PR>
__global__ void encode_kernel(BoxDesc b, int parity, int field, const double* __restrict__ src, int64_t n) {
  using TM = typename PR::TM;
  using TP = typename PR::TP;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int x, y, z;
    node_xyz(b, i, x, y, z);
    if (field == 0) {
      ((gptr<TP>)b.phi[parity])[phi_at(b, x, y, z)] = Enc<TP>::go(src[i], 0.f, 1.f);
    } else {
      const int k = field - 1;
      if (k < b.nmom)  // Q is not stored by the gradient closure
        ((gptr<TM>)b.mom[parity])[mom_at(b, k, x, y, z)] = Enc<TM>::go(src[i], b.enc_off[k], b.enc_scale[k]);
    }
  }
}

template <class PR>
__global__ void decode_kernel(BoxDesc b, int parity, int field, double* __restrict__ dst, int64_t n) {
  using TM = typename PR::TM;
  using TP = typename PR::TP;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int x, y, z;
    node_xyz(b, i, x, y, z);
    if (field == 0) {
      dst[i] = dec<double>(((gptr<const TP>)b.phi[parity])[phi_at(b, x, y, z)], 0.f, 1.f);
    } else {
      const int k = field - 1;
      dst[i] = k < b.nmom ? dec<double>(((gptr<const TM>)b.mom[parity])[mom_at(b, k, x, y, z)], b.enc_off[k], b.enc_inv[k])
                          : 0.0;
    }
  }
}

template <class PR>
__global__ void gather_kernel(BoxDesc b, int parity, const int64_t* __restrict__ idx, int64_t n,
                              double* __restrict__ out) {
  using TM = typename PR::TM;
  using TP = typename PR::TP;
  for (int64_t j = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; j < n;
       j += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int x, y, z;
    node_xyz(b, idx[j], x, y, z);
    out[j] = dec<double>(((gptr<const TP>)b.phi[parity])[phi_at(b, x, y, z)], 0.f, 1.f);
    for (int k = 0; k < 10; ++k)
      out[(k + 1) * n + j] = k < b.nmom ? dec<double>(((gptr<const TM>)b.mom[parity])[mom_at(b, k, x, y, z)],
                                                      b.enc_off[k], b.enc_inv[k])
                                        : 0.0;
  }
}

// Node quantities needed by the observables and diagnostics, in FP64 from
// the decoded state: rho, u = J + a/2, p = rho cs^2 p*.
template <class PR>
__device__ void node_obs(const BoxDesc& b, int parity, int x, int y, int z, double& rho, double u[3],
                         double& phi, double& p, double& pstar, bool& finite) {
  using TM = typename PR::TM;
  using TP = typename PR::TP;
  const int nx = b.nx, ny = b.ny, nz = b.nz;
  const gptr<const TP> fphi = (gptr<const TP>)b.phi[parity];
  const gptr<const TM> fmom = (gptr<const TM>)b.mom[parity];
  // loads without a per-moment runtime test (see diag_partial_kernel): the
  // closure's moment count selects one of two unrolled blocks
  double m[10];
  finite = true;
  auto load_moments = [&](auto nm) {
    constexpr int NMOM = decltype(nm)::value;
#pragma unroll
    for (int k = 0; k < 10; ++k) m[k] = 0.0;
#pragma unroll
    for (int k = 0; k < NMOM; ++k) {
      m[k] = dec<double>(fmom[mom_at(b, k, x, y, z)], b.enc_off[k], b.enc_inv[k]);
      finite = finite && isfinite(m[k]);
    }
  };
  if (b.nmom == 4) load_moments(std::integral_constant<int, 4>{});
  else load_moments(std::integral_constant<int, 10>{});
  phi = dec<double>(fphi[phi_at(b, x, y, z)], 0.f, 1.f);
  finite = finite && isfinite(phi);
  // neighbour coordinates per axis (wrap or mirror) and wall-crossing flags,
  // resolved once: xs[c + 1], ks_x[c + 1] for c = -1, 0, 1
  int xs[3], ys[3], zs[3], kxs[3], kys[3], kzs[3];
  for (int c = -1; c <= 1; ++c) {
    xs[c + 1] = map_axis(x + c, nx, b.wall[0], kxs[c + 1]);
    ys[c + 1] = map_axis(y + c, ny, b.wall[1], kys[c + 1]);
    zs[c + 1] = map_axis(z + c, nz, b.wall[2], kzs[c + 1]);
  }
  double g[3] = {0, 0, 0}, lap = 0;
  for (int cz = -1; cz <= 1; ++cz)
    for (int cy = -1; cy <= 1; ++cy) {
      const gptr<const TP> row = fphi + phi_at(b, 0, ys[cy + 1], zs[cz + 1]);
      for (int cx = -1; cx <= 1; ++cx) {
        const double v = dec<double>(row[xs[cx + 1]], 0.f, 1.f);
        const double w = (cx ? 1.0 : 4.0) * (cy ? 1.0 : 4.0) * (cz ? 1.0 : 4.0) / 216.0;
        g[0] += 3.0 * w * cx * v;
        g[1] += 3.0 * w * cy * v;
        g[2] += 3.0 * w * cz * v;
        lap += 6.0 * w * (v - phi);
      }
    }
  const double phic = fmin(fmax(phi, 0.0), 1.0);
  rho = b.rho_g + phic * b.drho;
  const double nu = b.nu_g + phic * b.dnu;
  const double om = 1.0 / (3.0 * nu + 0.5);
  const double mu = b.beta4 * phi * (phi - 1.0) * (phi - 0.5) - b.kappa_mu * lap;
  const double P = m[0];
  double Q[3][3] = {{m[4], m[7], m[8]}, {m[7], m[5], m[9]}, {m[8], m[9], m[6]}};
  if (b.flags & 2) {
    // gradient closure: the viscous correction contracts -(cs^2/omega)(grad J + grad J^T),
    // J ghosts minus the mirrored value per wall crossed
    double gJ[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    const int64_t fstride = static_cast<int64_t>(ny) * b.pitch;  // one moment plane
    for (int cz = -1; cz <= 1; ++cz)
      for (int cy = -1; cy <= 1; ++cy) {
        const gptr<const TM> rowJ = fmom + mom_at(b, 1, 0, ys[cy + 1], zs[cz + 1]);
        for (int cx = -1; cx <= 1; ++cx) {
          const double sgn = ((kxs[cx + 1] + kys[cy + 1] + kzs[cz + 1]) & 1) ? -1.0 : 1.0;
          const double w = 3.0 * (cx ? 1.0 : 4.0) * (cy ? 1.0 : 4.0) * (cz ? 1.0 : 4.0) / 216.0;
          for (int a = 0; a < 3; ++a) {
            const double ja = sgn * dec<double>(rowJ[a * fstride + xs[cx + 1]], b.enc_off[1 + a], b.enc_inv[1 + a]);
            gJ[a][0] += w * cx * ja;
            gJ[a][1] += w * cy * ja;
            gJ[a][2] += w * cz * ja;
          }
        }
      }
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) Q[a][c] = -(1.0 / 3.0) / om * (gJ[a][c] + gJ[c][a]);
  }
  for (int a = 0; a < 3; ++a) {
    double qg = 0;
    for (int c = 0; c < 3; ++c) qg += Q[a][c] * g[c] * b.drho;
    const double F = mu * g[a] - P * (1.0 / 3.0) * b.drho * g[a] - 3.0 * nu * om * qg +
                     (rho - b.rho_ref) * b.grav[a];
    u[a] = m[1 + a] + 0.5 * F / rho;
  }
  pstar = P;
  p = rho * (1.0 / 3.0) * P;
}

template <class PR>
__global__ void __launch_bounds__(256) observable_kernel(BoxDesc b, int parity, int which, double* __restrict__ dst) {
  const int64_t n = static_cast<int64_t>(b.nx) * b.ny * b.nz;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int x, y, z;
    node_xyz(b, i, x, y, z);
    double rho, u[3], phi, p, ps;
    bool fin;
    node_obs<PR>(b, parity, x, y, z, rho, u, phi, p, ps, fin);
    double v = 0;
    switch (which) {
      case 0: v = rho; break;
      case 1: v = u[0]; break;
      case 2: v = u[1]; break;
      case 3: v = u[2]; break;
      case 4: v = phi; break;
      default: v = p; break;
    }
    dst[i] = v;
  }
}

// Diagnostics value layout (kDiagValues doubles):
//  0 sum phi | 1 sum p* | 2-4 sum rho u | 5 sum rho|u|^2/2 | 6 max|u|
//  7-9 sum phi x | 10-12 sum phi u | 13 sum (1-phi) | 14-16 sum (1-phi) x
//  17-19 sum (1-phi) u | 20 sum p (phi>=0.98) | 21 count | 22 sum p (phi<=0.02)
//  23 count | 24 nonfinite flag | 25-27 unused
constexpr int kDiagThreads = 256;
constexpr int kDiagWaves = kDiagThreads / 64;

__device__ inline double combine(int k, double a, double b) {
  if (k == 6 || k == 24) return a > b ? a : b;
  return a + b;
}

// Sum (max for the max-type values) over the 64 lanes of a wavefront by a
// butterfly of lane exchanges; lane 0 ends with the values combined in a fixed
// order, so the result does not depend on scheduling.
__device__ __forceinline__ double wave_combine(int k, double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = combine(k, v, __shfl_xor(v, off, 64));
  return v;
}

// x-y parts of the isotropic 27-point stencils on one plane of a field, at
// column (x, y) with neighbour columns xs[cx + 1], ys[cy + 1] (wrap / mirror
// already resolved): F[0] = s_x s_y f, F[1] = s_y d_x f, F[2] = s_x d_y f with
// s = (1, 4, 1) and d = (-1, 0, 1), F[3] = f at the column.  ld(xm, ym, cx, cy)
// returns the decoded value of the (mapped) neighbour column.
template <class Load>
__device__ __forceinline__ void diag_filter(const Load& ld, const int xs[3], const int ys[3], double F[4]) {
  double sx[3], dx[3];
  for (int cy = 0; cy < 3; ++cy) {
    const double l = ld(xs[0], ys[cy], 0, cy), c = ld(xs[1], ys[cy], 1, cy), h = ld(xs[2], ys[cy], 2, cy);
    sx[cy] = l + 4.0 * c + h;
    dx[cy] = h - l;
    if (cy == 1) F[3] = c;
  }
  F[0] = sx[0] + 4.0 * sx[1] + sx[2];
  F[1] = dx[0] + 4.0 * dx[1] + dx[2];
  F[2] = sx[2] - sx[0];
}

constexpr int kDiagZ = 64;  // planes per work unit of the diagnostics z-march

// One launch covers boxes box0 .. box0 + gridDim.y - 1 of the descriptor
// array; gridDim.x workgroups share each box and write one partial per value:
// partials[(blockIdx.y * gridDim.x + blockIdx.x) * kDiagValues + k].
// A work unit is one column (x, y) over up to kDiagZ planes; consecutive
// threads take consecutive x, so every load is coalesced.  Each thread keeps
// the x-y filtered phi planes z-1, z, z+1 in registers (and, for the gradient
// closure, those of J), so a node costs 9 loads and conversions of phi
// instead of the 27 of a direct stencil; the node quantities are those of
// node_obs in FP64: rho, u = J + a/2 with the full force, p = rho cs^2 p*.
template <class PR, bool GC>
__global__ void __launch_bounds__(kDiagThreads) diag_partial_kernel(const BoxDesc* __restrict__ boxes, int box0, int parity,
                                                                    double* __restrict__ partials) {
  using TM = typename PR::TM;
  using TP = typename PR::TP;
  __shared__ double red[kDiagWaves][kDiagValues];
  const BoxDesc& b = boxes[box0 + blockIdx.y];
  double acc[kDiagValues];
  for (int k = 0; k < kDiagValues; ++k) acc[k] = 0.0;
  const int nx = b.nx, ny = b.ny, nz = b.nz;
  const int64_t ncol = static_cast<int64_t>(nx) * ny;
  const int64_t units = ncol * ((nz + kDiagZ - 1) / kDiagZ);
  const gptr<const TP> fphi = (gptr<const TP>)b.phi[parity];
  const gptr<const TM> fmom = (gptr<const TM>)b.mom[parity];
  for (int64_t un = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; un < units;
       un += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t col = un % ncol;
    const int x = static_cast<int>(col % nx), y = static_cast<int>(col / nx);
    const int z0 = static_cast<int>(un / ncol) * kDiagZ, z1 = min(z0 + kDiagZ, nz);
    int xs[3], ys[3], kx[3], ky[3];
    for (int c = -1; c <= 1; ++c) {
      xs[c + 1] = map_axis(x + c, nx, b.wall[0], kx[c + 1]);
      ys[c + 1] = map_axis(y + c, ny, b.wall[1], ky[c + 1]);
    }
    // Raw (still encoded) phi of the 3 x 3 columns of the next plane and the
    // node's moments are loaded one plane ahead, so their memory latency
    // overlaps the node's arithmetic.  The moment count is a compile-time
    // constant: a per-moment runtime test would put each load in a basic
    // block of its own, and with 16- or 32-bit storage the conversion after
    // it would wait for that load before the next one is issued.
    constexpr int NMOM = GC ? 4 : 10;
    TP rph[9];
    TM rm[NMOM];
    auto issue_phi = [&](int q) {
      const int zq = map_axis(q, nz, b.wall[2]);
#pragma unroll
      for (int cy = 0; cy < 3; ++cy)
#pragma unroll
        for (int cx = 0; cx < 3; ++cx) rph[cy * 3 + cx] = fphi[phi_at(b, xs[cx], ys[cy], zq)];
    };
    auto issue_mom = [&](int zm) {
#pragma unroll
      for (int k = 0; k < NMOM; ++k) rm[k] = fmom[mom_at(b, k, x, y, zm)];
    };
    auto filter_phi = [&](double F[4]) {
      auto ld = [&](int, int, int cx, int cy) { return dec<double>(rph[cy * 3 + cx], 0.f, 1.f); };
      diag_filter(ld, xs, ys, F);
    };
    // gradient closure: filtered J of plane q (J ghosts: minus the mirrored
    // value per crossed wall)
    auto filter_J = [&](int q, double JF[3][4]) {
      int kz;
      const int zq = map_axis(q, nz, b.wall[2], kz);
      for (int a = 0; a < 3; ++a) {
        auto ldj = [&](int xm, int ym, int cx, int cy) {
          const double v = dec<double>(fmom[mom_at(b, 1 + a, xm, ym, zq)], b.enc_off[1 + a], b.enc_inv[1 + a]);
          return ((kx[cx] + ky[cy] + kz) & 1) ? -v : v;
        };
        diag_filter(ldj, xs, ys, JF[a]);
      }
    };
    double Fm[4], F0[4], Fn[4];
    double JFm[GC ? 3 : 1][4], JF0[GC ? 3 : 1][4], JFn[GC ? 3 : 1][4];
    issue_phi(z0 - 1);
    filter_phi(Fm);
    issue_phi(z0);
    filter_phi(F0);
    if constexpr (GC) {
      filter_J(z0 - 1, JFm);
      filter_J(z0, JF0);
    }
    issue_phi(z0 + 1);
    issue_mom(z0);
    for (int z = z0; z < z1; ++z) {
      filter_phi(Fn);  // plane z + 1
      if constexpr (GC) filter_J(z + 1, JFn);
      double m[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) m[k] = 0.0;
#pragma unroll
      for (int k = 0; k < NMOM; ++k) m[k] = dec<double>(rm[k], b.enc_off[k], b.enc_inv[k]);
      if (z + 1 < z1) {
        issue_phi(z + 2);
        issue_mom(z + 1);
      }
      const double phi = F0[3];
      const double g[3] = {(Fm[1] + 4.0 * F0[1] + Fn[1]) * (1.0 / 72.0), (Fm[2] + 4.0 * F0[2] + Fn[2]) * (1.0 / 72.0),
                           (Fn[0] - Fm[0]) * (1.0 / 72.0)};
      const double lap = (Fm[0] + 4.0 * F0[0] + Fn[0]) * (1.0 / 36.0) - 6.0 * phi;
      bool fin = isfinite(phi);
#pragma unroll
      for (int k = 0; k < NMOM; ++k) fin = fin && isfinite(m[k]);
      const double phic = fmin(fmax(phi, 0.0), 1.0);
      const double rho = b.rho_g + phic * b.drho;
      const double nu = b.nu_g + phic * b.dnu;
      const double om = 1.0 / (3.0 * nu + 0.5);
      const double mu = b.beta4 * phi * (phi - 1.0) * (phi - 0.5) - b.kappa_mu * lap;
      const double P = m[0];
      double Q[3][3] = {{m[4], m[7], m[8]}, {m[7], m[5], m[9]}, {m[8], m[9], m[6]}};
      if constexpr (GC) {
        double gJ[3][3];  // gJ[a][c] = d_c J_a
        for (int a = 0; a < 3; ++a) {
          gJ[a][0] = (JFm[a][1] + 4.0 * JF0[a][1] + JFn[a][1]) * (1.0 / 72.0);
          gJ[a][1] = (JFm[a][2] + 4.0 * JF0[a][2] + JFn[a][2]) * (1.0 / 72.0);
          gJ[a][2] = (JFn[a][0] - JFm[a][0]) * (1.0 / 72.0);
        }
        for (int a = 0; a < 3; ++a)
          for (int c = 0; c < 3; ++c) Q[a][c] = -(1.0 / 3.0) / om * (gJ[a][c] + gJ[c][a]);
      }
      double u[3];
      for (int a = 0; a < 3; ++a) {
        double qg = 0;
        for (int c = 0; c < 3; ++c) qg += Q[a][c] * g[c] * b.drho;
        const double F = mu * g[a] - P * (1.0 / 3.0) * b.drho * g[a] - 3.0 * nu * om * qg +
                         (rho - b.rho_ref) * b.grav[a];
        u[a] = m[1 + a] + 0.5 * F / rho;
      }
      const double p = rho * (1.0 / 3.0) * P;
      const double sp = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
      const double pos[3] = {double(x), double(y), double(z)};
      acc[0] += phi;
      acc[1] += P;
      for (int a = 0; a < 3; ++a) acc[2 + a] += rho * u[a];
      acc[5] += 0.5 * rho * sp;
      acc[6] = fmax(acc[6], sqrt(sp));
      for (int a = 0; a < 3; ++a) {
        acc[7 + a] += phi * pos[a];
        acc[10 + a] += phi * u[a];
        acc[14 + a] += (1.0 - phi) * pos[a];
        acc[17 + a] += (1.0 - phi) * u[a];
      }
      acc[13] += 1.0 - phi;
      if (phi >= 0.98) { acc[20] += p; acc[21] += 1.0; }
      if (phi <= 0.02) { acc[22] += p; acc[23] += 1.0; }
      if (!fin) acc[24] = 1.0;
      for (int k = 0; k < 4; ++k) {
        Fm[k] = F0[k];
        F0[k] = Fn[k];
      }
      if constexpr (GC)
        for (int a = 0; a < 3; ++a)
          for (int k = 0; k < 4; ++k) {
            JFm[a][k] = JF0[a][k];
            JF0[a][k] = JFn[a][k];
          }
    }
  }
  // wavefront reductions (unrolled: a runtime index into acc would move the
  // accumulators from registers to scratch memory), then the waves of the
  // workgroup in order through LDS
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kDiagValues; ++k) {
    const double v = wave_combine(k, acc[k]);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < kDiagValues) {
    const int k = threadIdx.x;
    double v = red[0][k];
    for (int w = 1; w < kDiagWaves; ++w) v = combine(k, v, red[w][k]);
    partials[(static_cast<int64_t>(blockIdx.y) * gridDim.x + blockIdx.x) * kDiagValues + k] = v;
  }
}

// One workgroup per box: each wave takes values k = wave, wave + 4, ...; its
// lanes combine the box's nblocks partials in a fixed stride order, then the
// lanes by a wavefront reduction.  out[box * kDiagValues + k].
__global__ void __launch_bounds__(kDiagThreads) diag_final_kernel(const double* __restrict__ partials, int nblocks,
                                                                  double* __restrict__ out) {
  const double* p = partials + static_cast<int64_t>(blockIdx.x) * nblocks * kDiagValues;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = wave; k < kDiagValues; k += kDiagWaves) {
    double a = 0.0;  // identity of both the sums and the maxima (|u| and the flag are >= 0)
    for (int i = lane; i < nblocks; i += 64) a = combine(k, a, p[static_cast<int64_t>(i) * kDiagValues + k]);
    a = wave_combine(k, a);
    if (lane == 0) out[blockIdx.x * kDiagValues + k] = a;
  }
}

// ---------------------------------------------------------------------------
// Fourth-order phase-field update (LBM_HIGH_ORDER_AC)
// ---------------------------------------------------------------------------
// The higher-order discretisation that Sec. II.A names as future work, with
// no scheme given there: the divergence, the Laplacian and the gradient
// inside the normal of the FTCS update are the Richardson combination
// (4 D1 - D2) / 3 of the isotropic D3Q27 stencil at spacing 1 (D1, neighbours
// x + c) and at spacing 2 (D2, neighbours x + 2c, the first derivative
// divided by 2, the Laplacian by 4).  The leading errors of D1 and D2 are
// isotropic and in the ratio 1 : 4, so the combination removes them.  The
// flow solver keeps the second-order stencils (the fused step is unchanged;
// its phi output is overwritten).  Two kernels, both reading level n:
//   ho_flux_kernel  per node: u = J + a/2 with the forces of Sec. II.C
//                   (node_obs, FP64) and S = phi (1 - phi) n4, n4 the unit
//                   fourth-order gradient; 6 doubles into b.aux;
//   ho_phase_kernel per node: phi' = phi - div4(phi u) + M lap4(phi)
//                   - (4M/W) div4(S), or u . grad4(phi) for the printed
//                   advection.  Neighbours beyond a wall are mirrored nodes,
//                   with u negated per crossed wall and the crossed
//                   components of S negated (the normal of the mirrored phi).

// phi of node (x, y, z), coordinates already inside the box
template <class PR>
__device__ __forceinline__ double phi_node(const BoxDesc& b, int parity, int x, int y, int z) {
  using TP = typename PR::TP;
  return dec<double>(((gptr<const TP>)b.phi[parity])[phi_at(b, x, y, z)], 0.f, 1.f);
}

template <class PR>
__global__ void __launch_bounds__(256) ho_flux_kernel(const BoxDesc* __restrict__ boxes, int box0, int parity) {
  const BoxDesc& b = boxes[box0 + blockIdx.y];
  const int64_t n = static_cast<int64_t>(b.nx) * b.ny * b.nz;
  double* aux = b.aux;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int x, y, z;
    node_xyz(b, i, x, y, z);
    double rho, u[3], phi, p, ps;
    bool fin;
    node_obs<PR>(b, parity, x, y, z, rho, u, phi, p, ps, fin);
    double g1[3] = {0, 0, 0}, g2[3] = {0, 0, 0};
    for (int cz = -1; cz <= 1; ++cz)
      for (int cy = -1; cy <= 1; ++cy)
        for (int cx = -1; cx <= 1; ++cx) {
          if (cx == 0 && cy == 0 && cz == 0) continue;
          const double w = (cx ? 1.0 : 4.0) * (cy ? 1.0 : 4.0) * (cz ? 1.0 : 4.0) / 216.0;
          const double v1 = phi_node<PR>(b, parity, map_axis(x + cx, b.nx, b.wall[0]), map_axis(y + cy, b.ny, b.wall[1]),
                                         map_axis(z + cz, b.nz, b.wall[2]));
          const double v2 = phi_node<PR>(b, parity, map_axis(x + 2 * cx, b.nx, b.wall[0]),
                                         map_axis(y + 2 * cy, b.ny, b.wall[1]), map_axis(z + 2 * cz, b.nz, b.wall[2]));
          const double c[3] = {double(cx), double(cy), double(cz)};
          for (int a = 0; a < 3; ++a) {
            g1[a] += 3.0 * w * c[a] * v1;
            g2[a] += 1.5 * w * c[a] * v2;
          }
        }
    double g[3];
    for (int a = 0; a < 3; ++a) g[a] = (4.0 * g1[a] - g2[a]) / 3.0;
    const double inv = 1.0 / (sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + 1e-12);
    const double pp = phi * (1.0 - phi);
    for (int a = 0; a < 3; ++a) {
      aux[a * n + i] = u[a];
      aux[(3 + a) * n + i] = pp * g[a] * inv;
    }
  }
}

template <class PR>
__global__ void __launch_bounds__(256) ho_phase_kernel(const BoxDesc* __restrict__ boxes, int box0, int parity) {
  using TP = typename PR::TP;
  const BoxDesc& b = boxes[box0 + blockIdx.y];
  const int nx = b.nx, ny = b.ny, nz = b.nz;
  const int64_t n = static_cast<int64_t>(nx) * ny * nz;
  const double* aux = b.aux;
  const bool literal = (b.flags & 1) != 0;
  const double kac = b.kappa_ac, mob = b.mobility;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int x, y, z;
    node_xyz(b, i, x, y, z);
    const double phi0 = phi_node<PR>(b, parity, x, y, z);
    double adv[2] = {0, 0}, shp[2] = {0, 0}, lap[2] = {0, 0}, g[2][3] = {{0, 0, 0}, {0, 0, 0}};
    for (int cz = -1; cz <= 1; ++cz)
      for (int cy = -1; cy <= 1; ++cy)
        for (int cx = -1; cx <= 1; ++cx) {
          if (cx == 0 && cy == 0 && cz == 0) continue;
          const double w = (cx ? 1.0 : 4.0) * (cy ? 1.0 : 4.0) * (cz ? 1.0 : 4.0) / 216.0;
          const double c[3] = {double(cx), double(cy), double(cz)};
          for (int s = 1; s <= 2; ++s) {
            int kx, ky, kz;
            const int xm = map_axis(x + s * cx, nx, b.wall[0], kx);
            const int ym = map_axis(y + s * cy, ny, b.wall[1], ky);
            const int zm = map_axis(z + s * cz, nz, b.wall[2], kz);
            const int64_t j = (static_cast<int64_t>(zm) * ny + ym) * nx + xm;
            const double ph = phi_node<PR>(b, parity, xm, ym, zm);
            const double su = ((kx + ky + kz) & 1) ? -1.0 : 1.0;
            const double sn[3] = {kx ? -1.0 : 1.0, ky ? -1.0 : 1.0, kz ? -1.0 : 1.0};
            double uc = 0, sc = 0;
            for (int a = 0; a < 3; ++a) {
              uc += c[a] * aux[a * n + j];
              sc += c[a] * sn[a] * aux[(3 + a) * n + j];
            }
            const double wt = 3.0 * w / s;
            adv[s - 1] += wt * ph * su * uc;
            shp[s - 1] += wt * sc;
            lap[s - 1] += (6.0 * w / (s * s)) * (ph - phi0);
            for (int a = 0; a < 3; ++a) g[s - 1][a] += wt * c[a] * ph;
          }
        }
    auto four = [](const double* v) { return (4.0 * v[0] - v[1]) / 3.0; };
    double a_term;
    if (literal) {
      a_term = 0.0;
      for (int a = 0; a < 3; ++a) a_term += aux[a * n + i] * (4.0 * g[0][a] - g[1][a]) / 3.0;
    } else {
      a_term = four(adv);
    }
    const double phin = phi0 - a_term + mob * four(lap) - kac * four(shp);
    ((gptr<TP>)b.phi[1 - parity])[phi_at(b, x, y, z)] = Enc<TP>::go(phin, 0.f, 1.f);
  }
}

int grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return static_cast<int>(g);
}

}  // namespace

hipError_t launch_encode(int precision, const BoxDesc& box, int parity, int field, const double* d_src,
                         int64_t n, hipStream_t stream) {
  return dispatch(precision, [&](auto pr) {
    using PR = decltype(pr);
    hipLaunchKernelGGL((encode_kernel<PR>), dim3(grid_for(n, 256)), dim3(256), 0, stream, box, parity, field,
                       d_src, n);
    return hipGetLastError();
  });
}

hipError_t launch_decode(int precision, const BoxDesc& box, int parity, int field, double* d_dst, int64_t n,
                         hipStream_t stream) {
  return dispatch(precision, [&](auto pr) {
    using PR = decltype(pr);
    hipLaunchKernelGGL((decode_kernel<PR>), dim3(grid_for(n, 256)), dim3(256), 0, stream, box, parity, field,
                       d_dst, n);
    return hipGetLastError();
  });
}

hipError_t launch_gather(int precision, const BoxDesc& box, int parity, const int64_t* d_idx, int64_t n,
                         double* d_out, hipStream_t stream) {
  return dispatch(precision, [&](auto pr) {
    using PR = decltype(pr);
    hipLaunchKernelGGL((gather_kernel<PR>), dim3(grid_for(n, 256)), dim3(256), 0, stream, box, parity, d_idx, n,
                       d_out);
    return hipGetLastError();
  });
}

hipError_t launch_observable(int precision, const BoxDesc& box, int parity, int which, double* d_dst,
                             hipStream_t stream) {
  const int64_t n = static_cast<int64_t>(box.nx) * box.ny * box.nz;
  return dispatch(precision, [&](auto pr) {
    using PR = decltype(pr);
    hipLaunchKernelGGL((observable_kernel<PR>), dim3(grid_for(n, 256)), dim3(256), 0, stream, box, parity,
                       which, d_dst);
    return hipGetLastError();
  });
}

int high_order_blocks_per_box(int64_t max_nodes) {
  int64_t nb = (max_nodes + 256 * 4 - 1) / (256 * 4);
  return static_cast<int>(nb < 1 ? 1 : (nb > 8192 ? 8192 : nb));
}

hipError_t launch_high_order_phase(int precision, const BoxDesc* d_boxes, int box0, int nbox, int parity,
                                   int blocks_per_box, hipStream_t stream) {
  if (nbox <= 0 || blocks_per_box <= 0) return hipErrorInvalidValue;
  return dispatch(precision, [&](auto pr) {
    using PR = decltype(pr);
    hipLaunchKernelGGL((ho_flux_kernel<PR>), dim3(blocks_per_box, nbox), dim3(256), 0, stream, d_boxes, box0, parity);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((ho_phase_kernel<PR>), dim3(blocks_per_box, nbox), dim3(256), 0, stream, d_boxes, box0, parity);
    return hipGetLastError();
  });
}

int diag_blocks_per_box(int64_t max_nodes) {
  int64_t nb = (max_nodes + kDiagThreads * 16 - 1) / (kDiagThreads * 16);
  return static_cast<int>(nb < 1 ? 1 : (nb > kDiagBlocks ? kDiagBlocks : nb));
}

hipError_t launch_diagnostics(int precision, bool gc, const BoxDesc* d_boxes, int box0, int nbox, int parity,
                              int blocks_per_box, double* d_partials, double* d_out, hipStream_t stream) {
  if (nbox <= 0 || blocks_per_box <= 0) return hipErrorInvalidValue;
  hipError_t e = dispatch(precision, [&](auto pr) {
    using PR = decltype(pr);
    if (gc)
      hipLaunchKernelGGL((diag_partial_kernel<PR, true>), dim3(blocks_per_box, nbox), dim3(kDiagThreads), 0, stream,
                         d_boxes, box0, parity, d_partials);
    else
      hipLaunchKernelGGL((diag_partial_kernel<PR, false>), dim3(blocks_per_box, nbox), dim3(kDiagThreads), 0, stream,
                         d_boxes, box0, parity, d_partials);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(diag_final_kernel, dim3(nbox), dim3(kDiagThreads), 0, stream, d_partials, blocks_per_box, d_out);
  return hipGetLastError();
}

}  // namespace lbm
