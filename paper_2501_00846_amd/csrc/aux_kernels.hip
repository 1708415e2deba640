// Device code of liblbm.so beyond the fused step: encoding of host fields
// into the storage formats and back, sampled readback, the observables
// (rho, u, phi, p), the FP64 diagnostics reductions, and the two kernels of
// the fourth-order phase-field variant.  None of them runs in the step loop
// except the fourth-order kernels, and those only with LBM_HIGH_ORDER_AC.
#include <hip/hip_runtime.h>

#include <algorithm>
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
// Element index of moment k of node (x, y, z) in the moment array of element
// type TM.  FP64 / FP32: plane k of the node's z plane.  16-bit storage: the
// moments are kept in pairs, (P, Jx), (Jy, Jz), (Qxx, Qyy), (Qzz, Qxy),
// (Qxz, Qyz) (P, J only with the gradient closure), one 32-bit word per node
// and pair with the even field in the low half (little-endian: the lower
// element index).
template <class TM>
__device__ __forceinline__ int64_t mom_at(const BoxDesc& b, int k, int x, int y, int z) {
  if constexpr (sizeof(TM) == 2)
    return 2 * (((static_cast<int64_t>(z) * (b.nmom / 2) + k / 2) * b.ny + y) * b.pitch + x) + (k & 1);
  else
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
        ((gptr<TM>)b.mom[parity])[mom_at<TM>(b, k, x, y, z)] = Enc<TM>::go(src[i], b.enc_off[k], b.enc_scale[k]);
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
      dst[i] = k < b.nmom ? dec<double>(((gptr<const TM>)b.mom[parity])[mom_at<TM>(b, k, x, y, z)], b.enc_off[k], b.enc_inv[k])
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
      out[(k + 1) * n + j] = k < b.nmom ? dec<double>(((gptr<const TM>)b.mom[parity])[mom_at<TM>(b, k, x, y, z)],
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
      m[k] = dec<double>(fmom[mom_at<TM>(b, k, x, y, z)], b.enc_off[k], b.enc_inv[k]);
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
    for (int cz = -1; cz <= 1; ++cz)
      for (int cy = -1; cy <= 1; ++cy) {
        for (int cx = -1; cx <= 1; ++cx) {
          const double sgn = ((kxs[cx + 1] + kys[cy + 1] + kzs[cz + 1]) & 1) ? -1.0 : 1.0;
          const double w = 3.0 * (cx ? 1.0 : 4.0) * (cy ? 1.0 : 4.0) * (cz ? 1.0 : 4.0) / 216.0;
          for (int a = 0; a < 3; ++a) {
            const double ja = sgn * dec<double>(fmom[mom_at<TM>(b, 1 + a, xs[cx + 1], ys[cy + 1], zs[cz + 1])],
                                                b.enc_off[1 + a], b.enc_inv[1 + a]);
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
      for (int k = 0; k < NMOM; ++k) rm[k] = fmom[mom_at<TM>(b, k, x, y, zm)];
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
          const double v = dec<double>(fmom[mom_at<TM>(b, 1 + a, xm, ym, zq)], b.enc_off[1 + a], b.enc_inv[1 + a]);
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
//   ho_flux_kernel  per node: u = J + a/2 with the forces of Sec. II.C (in
//                   FP64, as the diagnostics compute it) and S = phi (1 - phi)
//                   n4, n4 the unit fourth-order gradient; 6 values in the
//                   phi storage type into b.aux;
//   ho_phase_kernel per node, in the phi storage type's precision:
//                   phi' = phi - div4(phi u) + M lap4(phi)
//                   - (4M/W) div4(S), or u . grad4(phi) for the printed
//                   advection.  Neighbours beyond a wall are mirrored nodes,
//                   with u negated per crossed wall and the crossed
//                   components of S negated (the normal of the mirrored phi).
// Both march along z.  D1 and D2 are each separable: weights (1, 4, 1) and
// (-1, 0, 1) per axis, at taps +-1 or +-2.  A kernel filters every plane it
// meets in x and y once, keeps the filtered planes z-2 .. z+2 in registers,
// and combines them along z.

constexpr int kHoZ = 64;  // planes per work unit / tile of the z-marches

// u and S = phi (1 - phi) n4 per node into b.aux (6 compact planes in the
// phi storage type; with WS false u only, 3 planes, for the finer phase
// grid).  Work units: one
// column (x, y) over up to kHoZ planes, consecutive threads on consecutive x.
// Per plane the thread filters phi over its 3 x 3 columns at spacing 1 (F1)
// and at spacing 2 (F2), the raw values of the next planes and the node's
// moments loaded one plane ahead.
template <class PR, bool GC, bool WS>
__global__ void __launch_bounds__(256) ho_flux_kernel(const BoxDesc* __restrict__ boxes, int box0, int parity) {
  using TM = typename PR::TM;
  using TP = typename PR::TP;
  const BoxDesc& b = boxes[box0 + blockIdx.y];
  const int nx = b.nx, ny = b.ny, nz = b.nz;
  const int64_t n = static_cast<int64_t>(nx) * ny * nz;
  const int64_t ncol = static_cast<int64_t>(nx) * ny;
  const int64_t units = ncol * ((nz + kHoZ - 1) / kHoZ);
  const gptr<const TP> fphi = (gptr<const TP>)b.phi[parity];
  const gptr<const TM> fmom = (gptr<const TM>)b.mom[parity];
  TP* __restrict__ aux = static_cast<TP*>(b.aux);
  constexpr int NMOM = GC ? 4 : 10;
  for (int64_t un = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; un < units;
       un += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t col = un % ncol;
    const int x = static_cast<int>(col % nx), y = static_cast<int>(col / nx);
    const int z0 = static_cast<int>(un / ncol) * kHoZ, z1 = min(z0 + kHoZ, nz);
    int xs[3], ys[3], kx[3], ky[3], xs2[3], ys2[3];
    for (int c = -1; c <= 1; ++c) {
      xs[c + 1] = map_axis(x + c, nx, b.wall[0], kx[c + 1]);
      ys[c + 1] = map_axis(y + c, ny, b.wall[1], ky[c + 1]);
      xs2[c + 1] = map_axis(x + 2 * c, nx, b.wall[0]);
      ys2[c + 1] = map_axis(y + 2 * c, ny, b.wall[1]);
    }
    TP r1[9], r2[9];
    TM rm[NMOM];
    auto issue1 = [&](int q) {
      const int zq = map_axis(q, nz, b.wall[2]);
#pragma unroll
      for (int k = 0; k < 9; ++k) r1[k] = fphi[phi_at(b, xs[k % 3], ys[k / 3], zq)];
    };
    auto issue2 = [&](int q) {
      const int zq = map_axis(q, nz, b.wall[2]);
#pragma unroll
      for (int k = 0; k < 9; ++k) r2[k] = fphi[phi_at(b, xs2[k % 3], ys2[k / 3], zq)];
    };
    auto issue_mom = [&](int zm) {
#pragma unroll
      for (int k = 0; k < NMOM; ++k) rm[k] = fmom[mom_at<TM>(b, k, x, y, zm)];
    };
    auto filt = [&](const TP* r, double F[4]) {
      auto ld = [&](int, int, int cx, int cy) { return dec<double>(r[cy * 3 + cx], 0.f, 1.f); };
      diag_filter(ld, xs, ys, F);
    };
    auto filter_J = [&](int q, double JF[3][4]) {
      int kz;
      const int zq = map_axis(q, nz, b.wall[2], kz);
      for (int a = 0; a < 3; ++a) {
        auto ldj = [&](int xm, int ym, int cx, int cy) {
          const double v = dec<double>(fmom[mom_at<TM>(b, 1 + a, xm, ym, zq)], b.enc_off[1 + a], b.enc_inv[1 + a]);
          return ((kx[cx] + ky[cy] + kz) & 1) ? -v : v;
        };
        diag_filter(ldj, xs, ys, JF[a]);
      }
    };
    // F1 of planes z-1, z, z+1; F2 of planes z-2 .. z+2
    double F1[3][4], F2[5][4] = {};
    double JFm[GC ? 3 : 1][4], JF0[GC ? 3 : 1][4], JFn[GC ? 3 : 1][4];
    issue1(z0 - 1);
    filt(r1, F1[0]);
    issue1(z0);
    filt(r1, F1[1]);
    if constexpr (WS) {
      for (int k = 0; k < 4; ++k) {
        issue2(z0 - 2 + k);
        filt(r2, F2[k]);
      }
    }
    if constexpr (GC) {
      filter_J(z0 - 1, JFm);
      filter_J(z0, JF0);
    }
    issue1(z0 + 1);
    if constexpr (WS) issue2(z0 + 2);
    issue_mom(z0);
    for (int z = z0; z < z1; ++z) {
      filt(r1, F1[2]);  // plane z + 1
      if constexpr (WS) filt(r2, F2[4]);  // plane z + 2
      if constexpr (GC) filter_J(z + 1, JFn);
      double m[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) m[k] = 0.0;
#pragma unroll
      for (int k = 0; k < NMOM; ++k) m[k] = dec<double>(rm[k], b.enc_off[k], b.enc_inv[k]);
      if (z + 1 < z1) {
        issue1(z + 2);
        if constexpr (WS) issue2(z + 3);
        issue_mom(z + 1);
      }
      const double phi = F1[1][3];
      const double g[3] = {(F1[0][1] + 4.0 * F1[1][1] + F1[2][1]) * (1.0 / 72.0),
                           (F1[0][2] + 4.0 * F1[1][2] + F1[2][2]) * (1.0 / 72.0), (F1[2][0] - F1[0][0]) * (1.0 / 72.0)};
      const double lap = (F1[0][0] + 4.0 * F1[1][0] + F1[2][0]) * (1.0 / 36.0) - 6.0 * phi;
      const double g2[3] = {(F2[0][1] + 4.0 * F2[2][1] + F2[4][1]) * (1.0 / 144.0),
                            (F2[0][2] + 4.0 * F2[2][2] + F2[4][2]) * (1.0 / 144.0),
                            (F2[4][0] - F2[0][0]) * (1.0 / 144.0)};
      // u = J + a/2 with the second-order forces of Sec. II.C (node_obs)
      const double phic = fmin(fmax(phi, 0.0), 1.0);
      const double rho = b.rho_g + phic * b.drho;
      const double nu = b.nu_g + phic * b.dnu;
      const double om = 1.0 / (3.0 * nu + 0.5);
      const double mu = b.beta4 * phi * (phi - 1.0) * (phi - 0.5) - b.kappa_mu * lap;
      const double P = m[0];
      double Q[3][3] = {{m[4], m[7], m[8]}, {m[7], m[5], m[9]}, {m[8], m[9], m[6]}};
      if constexpr (GC) {
        double gJ[3][3];
        for (int a = 0; a < 3; ++a) {
          gJ[a][0] = (JFm[a][1] + 4.0 * JF0[a][1] + JFn[a][1]) * (1.0 / 72.0);
          gJ[a][1] = (JFm[a][2] + 4.0 * JF0[a][2] + JFn[a][2]) * (1.0 / 72.0);
          gJ[a][2] = (JFn[a][0] - JFm[a][0]) * (1.0 / 72.0);
        }
        for (int a = 0; a < 3; ++a)
          for (int c = 0; c < 3; ++c) Q[a][c] = -(1.0 / 3.0) / om * (gJ[a][c] + gJ[c][a]);
      }
      double g4[3];
      for (int a = 0; a < 3; ++a) g4[a] = (4.0 * g[a] - g2[a]) / 3.0;
      const double inv = 1.0 / (sqrt(g4[0] * g4[0] + g4[1] * g4[1] + g4[2] * g4[2]) + 1e-12);
      const double pp = phi * (1.0 - phi);
      const int64_t i = (static_cast<int64_t>(z) * ny + y) * nx + x;
      for (int a = 0; a < 3; ++a) {
        double qg = 0;
        for (int c = 0; c < 3; ++c) qg += Q[a][c] * g[c] * b.drho;
        const double F = mu * g[a] - P * (1.0 / 3.0) * b.drho * g[a] - 3.0 * nu * om * qg +
                         (rho - b.rho_ref) * b.grav[a];
        aux[a * n + i] = static_cast<TP>(m[1 + a] + 0.5 * F / rho);
        if constexpr (WS) aux[(3 + a) * n + i] = static_cast<TP>(pp * g4[a] * inv);
      }
      for (int k = 0; k < 4; ++k) {
        F1[0][k] = F1[1][k];
        F1[1][k] = F1[2][k];
        if constexpr (WS)
          for (int p = 0; p < 4; ++p) F2[p][k] = F2[p + 1][k];
      }
      if constexpr (GC)
        for (int a = 0; a < 3; ++a)
          for (int k = 0; k < 4; ++k) {
            JFm[a][k] = JF0[a][k];
            JF0[a][k] = JFn[a][k];
          }
    }
  }
}

// The phase update.  A workgroup of 256 threads owns a tile of kHoTX x kHoTY
// output columns and marches it over up to kHoZ planes.  Per plane it stages,
// with a two-column halo, the flux G = phi u + (4M/W) S (only (4M/W) S for
// the printed advection) and phi in LDS, ghost rules applied as the values
// are staged; each thread then filters its column in x and y at spacings 1
// and 2 from LDS and keeps the filtered values of planes z-2 .. z+2 in
// registers.  With plane z+2 staged, output plane z is complete.
constexpr int kHoTX = 32, kHoTY = 8;
constexpr int kHoPX = kHoTX + 4, kHoPY = kHoTY + 4, kHoNP = kHoPX * kHoPY;
constexpr int kHoPer = (kHoNP + 255) / 256;  // staged elements per thread

// LIT: the boxes advect phi with the printed u . grad(phi) (every box of a
// launch alike); only then are the x and y differences of phi carried.
template <class PR, bool LIT>
__global__ void __launch_bounds__(256) ho_phase_kernel(const BoxDesc* __restrict__ boxes, int box0, int parity) {
  using TP = typename PR::TP;
  using RA = TP;  // arithmetic: FP64 for FP64 storage, FP32 otherwise
  constexpr int NV = LIT ? 6 : 4;  // filtered values per plane
  __shared__ RA sG[3][kHoNP];
  __shared__ RA sP[kHoNP];
  const BoxDesc& b = boxes[box0 + blockIdx.y];
  const int nx = b.nx, ny = b.ny, nz = b.nz;
  const int ntx = (nx + kHoTX - 1) / kHoTX, nty = (ny + kHoTY - 1) / kHoTY;
  const int tiles = ntx * nty * ((nz + kHoZ - 1) / kHoZ);
  if (static_cast<int>(blockIdx.x) >= tiles) return;  // uniform: boxes have different tile counts
  const int t = blockIdx.x;
  const int x0 = (t % ntx) * kHoTX, y0 = ((t / ntx) % nty) * kHoTY, z0 = (t / (ntx * nty)) * kHoZ;
  const int z1 = min(z0 + kHoZ, nz);
  const int64_t n = static_cast<int64_t>(nx) * ny * nz;
  const TP* __restrict__ aux = static_cast<const TP*>(b.aux);
  const gptr<const TP> fphi = (gptr<const TP>)b.phi[parity];
  const RA kac = static_cast<RA>(b.kappa_ac), mob = static_cast<RA>(b.mobility);
  const int tid = threadIdx.x;
  const int lx = tid % kHoTX, ly = tid / kHoTX;
  const int x = x0 + lx, y = y0 + ly;
  const bool active = x < nx && y < ny;
  // staged elements of this thread: mapped column and crossing flags
  int ecol[kHoPer], ex[kHoPer], ey[kHoPer], ekx[kHoPer], eky[kHoPer];
  for (int j = 0; j < kHoPer; ++j) {
    const int e = tid + 256 * j;
    const int ee = e < kHoNP ? e : 0;
    ex[j] = map_axis(x0 - 2 + ee % kHoPX, nx, b.wall[0], ekx[j]);
    ey[j] = map_axis(y0 - 2 + ee / kHoPX, ny, b.wall[1], eky[j]);
    ecol[j] = ey[j] * nx + ex[j];
  }
  // the next plane's staged values, loaded into registers a plane ahead:
  // raw phi, u and S of each element, and the plane's z crossing
  TP nph[kHoPer];
  TP nu[kHoPer][3], ns[kHoPer][3];
  int nkz = 0;
  auto load = [&](int q) {
    const int zq = map_axis(q, nz, b.wall[2], nkz);
    for (int j = 0; j < kHoPer; ++j) {  // elements past kHoNP load element 0 (never committed)
      const int64_t i = static_cast<int64_t>(zq) * nx * ny + ecol[j];
      nph[j] = fphi[phi_at(b, ex[j], ey[j], zq)];
      for (int a = 0; a < 3; ++a) {
        if constexpr (!LIT) nu[j][a] = aux[a * n + i];
        ns[j][a] = aux[(3 + a) * n + i];
      }
    }
  };
  auto commit = [&]() {
    for (int j = 0; j < kHoPer; ++j) {
      const int e = tid + 256 * j;
      if (e >= kHoNP) continue;
      const RA ph = dec<RA>(nph[j], 0.f, 1.f);
      const RA su = ((ekx[j] + eky[j] + nkz) & 1) ? RA(-1) : RA(1);
      const RA r[3] = {ekx[j] ? RA(-1) : RA(1), eky[j] ? RA(-1) : RA(1), nkz ? RA(-1) : RA(1)};
      for (int a = 0; a < 3; ++a) {
        const RA adv = LIT ? RA(0) : su * ph * nu[j][a];
        sG[a][e] = adv + kac * (r[a] * ns[j][a]);
      }
      sP[e] = ph;
    }
  };
  // filtered values of one plane at this thread's column, spacing s:
  // v[0] = sum_cy w(cy) (Gx(+s, cy) - Gx(-s, cy)), v[1] likewise for Gy
  // along y, v[2] = sum w w Gz, v[3] = sum w w phi, v[4], v[5] = the
  // x and y differences of phi (printed advection)
  auto filt = [&](int s, RA* v) {
    const int c0 = (ly + 2) * kHoPX + lx + 2;
    RA hx = 0, hy = 0, hz = 0, L = 0, dx = 0, dy = 0;
    for (int cy = -1; cy <= 1; ++cy)
      for (int cx = -1; cx <= 1; ++cx) {
        const RA w = RA((cx ? 1 : 4) * (cy ? 1 : 4));
        const int e = c0 + s * (cy * kHoPX + cx);
        hx += w * cx * sG[0][e];
        hy += w * cy * sG[1][e];
        hz += w * sG[2][e];
        L += w * sP[e];
        if constexpr (LIT) {
          dx += w * cx * sP[e];
          dy += w * cy * sP[e];
        }
      }
    v[0] = hx;
    v[1] = hy;
    v[2] = hz;
    v[3] = L;
    if constexpr (LIT) {
      v[4] = dx;
      v[5] = dy;
    }
  };
  // rings of the last staged planes: V1 at spacing 1 for planes z-1 .. z+2
  // (index 0 .. 3; z-1, z, z+1 used), V2 at spacing 2 for planes z-2 .. z+2
  // (index 0 .. 4; z-2, z, z+2 used); PC: phi at the column for planes z,
  // z+1, z+2
  RA V1[4][NV], V2[5][NV], PC[3];
  load(z0 - 2);
  for (int q = z0 - 2; q <= z1 + 1; ++q) {
    commit();
    __syncthreads();
    if (q < z1 + 1) load(q + 1);  // in flight while this plane is filtered and used
    const int k1 = q - (z0 - 2);  // planes staged so far - 1
    {
      RA v1[NV], v2[NV];
      filt(1, v1);
      filt(2, v2);
      const RA pc = sP[(ly + 2) * kHoPX + lx + 2];
      // shift the rings and append plane q
      for (int k = 0; k < NV; ++k) {
        for (int p = 0; p < 3; ++p) V1[p][k] = V1[p + 1][k];
        for (int p = 0; p < 4; ++p) V2[p][k] = V2[p + 1][k];
        V1[3][k] = v1[k];
        V2[4][k] = v2[k];
      }
      PC[0] = PC[1];
      PC[1] = PC[2];
      PC[2] = pc;
    }
    __syncthreads();
    if (k1 < 4) continue;  // output plane z = q - 2 needs planes z-2 .. z+2
    const int z = q - 2;
    if (!active) continue;
    const RA phi = PC[0];
    const RA div1 = (V1[0][0] + RA(4) * V1[1][0] + V1[2][0]) + (V1[0][1] + RA(4) * V1[1][1] + V1[2][1]) +
                    (V1[2][2] - V1[0][2]);
    const RA div2 = (V2[0][0] + RA(4) * V2[2][0] + V2[4][0]) + (V2[0][1] + RA(4) * V2[2][1] + V2[4][1]) +
                    (V2[4][2] - V2[0][2]);
    const RA lap1 = (V1[0][3] + RA(4) * V1[1][3] + V1[2][3]) * RA(1.0 / 36.0) - RA(6) * phi;
    const RA lap2 = (V2[0][3] + RA(4) * V2[2][3] + V2[4][3]) * RA(1.0 / 144.0) - RA(1.5) * phi;
    const RA div4 = (RA(4) * div1 * RA(1.0 / 72.0) - div2 * RA(1.0 / 144.0)) / RA(3);
    const RA lap4 = (RA(4) * lap1 - lap2) / RA(3);
    RA adv = 0;
    if constexpr (LIT) {
      const int64_t i = (static_cast<int64_t>(z) * ny + y) * nx + x;
      const RA g1[3] = {(V1[0][4] + RA(4) * V1[1][4] + V1[2][4]) * RA(1.0 / 72.0),
                        (V1[0][5] + RA(4) * V1[1][5] + V1[2][5]) * RA(1.0 / 72.0),
                        (V1[2][3] - V1[0][3]) * RA(1.0 / 72.0)};
      const RA g2[3] = {(V2[0][4] + RA(4) * V2[2][4] + V2[4][4]) * RA(1.0 / 144.0),
                        (V2[0][5] + RA(4) * V2[2][5] + V2[4][5]) * RA(1.0 / 144.0),
                        (V2[4][3] - V2[0][3]) * RA(1.0 / 144.0)};
      for (int a = 0; a < 3; ++a) adv += aux[a * n + i] * (RA(4) * g1[a] - g2[a]) / RA(3);
    }
    const RA phin = phi - adv - div4 + mob * lap4;
    ((gptr<TP>)b.phi[1 - parity])[phi_at(b, x, y, z)] = Enc<TP>::go(phin, 0.f, 1.f);
  }
}

// ---------------------------------------------------------------------------
// Finer phase-field grid (LBM_FINE_PHASE)
// ---------------------------------------------------------------------------
// The finer grid that Sec. II.A names as future work, with no scheme given
// there.  The phase field lives on a grid refined by 2 per axis, cell
// centred: coarse node i has the fine nodes 2i and 2i + 1 at i - 1/4 and
// i + 1/4, spacing h = 1/2.  The flow solver (the fused step, unchanged)
// reads the coarse phi, which is kept equal to the mean of the 8 fine nodes
// of its cell.  After the fused step of a step, reading level n:
//   ho_flux_kernel<PR, GC, false>  coarse u = J + a/2 into b.aux;
//   fine_step_kernel   phi_f' = phi_f - div_h G + M lap_h phi_f into the other
//                      fine buffer (the isotropic stencils of Sec. II.C
//                      divided by h and h^2), with the flux
//                      G = phi u_f + (4M/W) phi (1 - phi) n computed in LDS
//                      where it is used, u_f the trilinear interpolation of
//                      the coarse u, n from the isotropic gradient at
//                      spacing h;
//   fine_restrict_kernel  coarse phi' = mean of the 8 fine nodes, over the
//                      fused step's phi output.
// A ghost node of the fine grid beyond a wall takes the flux of its mirror
// node with u negated per crossed wall and the crossed components of the
// normal negated (the normal of the mirrored phi); the divergence then
// telescopes, and the fine phase mass is conserved.

__device__ __forceinline__ int64_t fine_at(const BoxDesc& b, int x, int y, int z) {
  return (static_cast<int64_t>(z) * (2 * b.ny) + y) * (2 * b.nx) + x;
}

// Trilinear interpolation at fine node (X, Y, Z) of a coarse field read by
// ld(x, y, z) at mapped coordinates (a coarse ghost beyond a wall takes the
// mirrored value): per axis coarse node X >> 1 with weight 3/4 and its
// neighbour towards the fine node (X even: below, odd: above) with weight 1/4.
template <class Load>
__device__ __forceinline__ double interp_fine(const BoxDesc& b, int X, int Y, int Z, const Load& ld) {
  int cx[2], cy[2], cz[2];
  cx[0] = X >> 1;
  cy[0] = Y >> 1;
  cz[0] = Z >> 1;
  cx[1] = map_axis(cx[0] + ((X & 1) ? 1 : -1), b.nx, b.wall[0]);
  cy[1] = map_axis(cy[0] + ((Y & 1) ? 1 : -1), b.ny, b.wall[1]);
  cz[1] = map_axis(cz[0] + ((Z & 1) ? 1 : -1), b.nz, b.wall[2]);
  double s = 0.0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const double w = (dx ? 0.25 : 0.75) * (dy ? 0.25 : 0.75) * (dz ? 0.25 : 0.75);
        s += w * ld(cx[dx], cy[dy], cz[dz]);
      }
  return s;
}

// fine phi of buffer s from the coarse phi of buffer s (initialisation)
template <class PR>
__global__ void fine_prolong_kernel(BoxDesc b, int s) {
  using TP = typename PR::TP;
  const int fx = 2 * b.nx, fy = 2 * b.ny;
  const int64_t nf = static_cast<int64_t>(fx) * fy * (2 * b.nz);
  const gptr<const TP> cphi = (gptr<const TP>)b.phi[s];
  const gptr<TP> fphi = (gptr<TP>)b.fphi[s];
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < nf;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int X = static_cast<int>(i % fx), Y = static_cast<int>((i / fx) % fy), Z = static_cast<int>(i / fx / fy);
    auto ld = [&](int x, int y, int z) { return dec<double>(cphi[phi_at(b, x, y, z)], 0.f, 1.f); };
    fphi[i] = Enc<TP>::go(interp_fine(b, X, Y, Z, ld), 0.f, 1.f);
  }
}

// coarse phi of buffer s = mean of the 8 fine nodes of each cell (fine buffer s)
template <class PR>
__global__ void __launch_bounds__(256) fine_restrict_kernel(const BoxDesc* __restrict__ boxes, int box0, int s) {
  using TP = typename PR::TP;
  const BoxDesc& b = boxes[box0 + blockIdx.y];
  const int64_t n = static_cast<int64_t>(b.nx) * b.ny * b.nz;
  const gptr<const TP> fphi = (gptr<const TP>)b.fphi[s];
  const gptr<TP> cphi = (gptr<TP>)b.phi[s];
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int x, y, z;
    node_xyz(b, i, x, y, z);
    double sum = 0.0;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) sum += dec<double>(fphi[fine_at(b, 2 * x + dx, 2 * y + dy, 2 * z + dz)], 0.f, 1.f);
    cphi[phi_at(b, x, y, z)] = Enc<TP>::go(0.125 * sum, 0.f, 1.f);
  }
}

template <class PR>
__global__ void fine_encode_kernel(BoxDesc b, int s, const double* __restrict__ src, int64_t n) {
  using TP = typename PR::TP;
  const gptr<TP> fphi = (gptr<TP>)b.fphi[s];
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    fphi[i] = Enc<TP>::go(src[i], 0.f, 1.f);
}

template <class PR>
__global__ void fine_decode_kernel(BoxDesc b, int s, double* __restrict__ dst, int64_t n) {
  using TP = typename PR::TP;
  const gptr<const TP> fphi = (gptr<const TP>)b.fphi[s];
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = dec<double>(fphi[i], 0.f, 1.f);
}

template <class PR>
__global__ void fine_gather_kernel(BoxDesc b, int s, const int64_t* __restrict__ idx, int64_t n,
                                   double* __restrict__ out) {
  using TP = typename PR::TP;
  const gptr<const TP> fphi = (gptr<const TP>)b.fphi[s];
  for (int64_t j = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; j < n;
       j += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[j] = dec<double>(fphi[idx[j]], 0.f, 1.f);
}

// The fine step phi_f' = phi_f - div_h G + M lap_h phi_f, with the flux
// G = phi u_f + (4M/W) phi (1 - phi) n computed where it is used.  A
// workgroup of 512 threads owns a tile of kFsTX x kFsTY fine columns and
// marches it over up to kHoZ planes; each of its first kFsGX x kFsGY threads
// owns one column of the flux region, the tile grown by one column.  Per
// staged plane r:
//   - the fine phi of the tile grown by two columns, continued across the
//     boundary (mirrored beyond a wall, wrapped on a periodic axis), goes to
//     LDS; each thread filters its column in x and y and keeps the filtered
//     planes r-3 .. r in registers;
//   - each thread computes the flux of plane r-1 at its column into LDS;
//   - after a barrier the tile's threads filter that flux plane in x and y
//     and keep the flux planes r-3 .. r-1 in registers, which completes
//     output plane r-2.
// On the continued phi field the gradient at a ghost node is the mirror
// node's with the crossed components negated, as the ghost rule asks.  The
// velocity is the trilinear interpolation of the coarse u continued as an
// odd field (minus the mirror value beyond a wall), which at a ghost node
// equals minus the interpolation at its mirror node.  Each coarse plane the
// tile needs is staged in LDS once (kFsUX x kFsUY coarse columns), loaded one
// fine plane ahead of its first use; every thread keeps the x-y bilinear sums
// of coarse planes c - 1, c, c + 1 around its flux plane in registers.  The
// staged loads of the next fine plane are issued before the current one is
// filtered.
constexpr int kFsThreads = 512;
constexpr int kFsTX = 32, kFsTY = 13;  // output columns of a tile (kFsTX even)
constexpr int kFsGX = kFsTX + 2, kFsGY = kFsTY + 2, kFsGN = kFsGX * kFsGY;  // flux region
constexpr int kFsPX = kFsTX + 4, kFsPY = kFsTY + 4, kFsPN = kFsPX * kFsPY;  // staged phi
// coarse columns under the flux region: fine X in [x0 - 1, x0 + kFsTX] needs
// coarse cells (X >> 1) - 1 .. (X >> 1) + 1, at most kFsTX / 2 + 4 of them
// for even x0, and (kFsTY + 1) / 2 + 3 in y for any y0
constexpr int kFsUX = kFsTX / 2 + 4, kFsUY = (kFsTY + 1) / 2 + 3, kFsUN = kFsUX * kFsUY;
static_assert(kFsGN <= kFsThreads, "one flux column per thread");
static_assert(kFsTX % 2 == 0, "tiles start at even fine x");

__host__ __device__ inline int fine_step_tiles(int nx, int ny, int nz) {
  return ((2 * nx + kFsTX - 1) / kFsTX) * ((2 * ny + kFsTY - 1) / kFsTY) * ((2 * nz + kHoZ - 1) / kHoZ);
}

template <class PR>
__global__ void __launch_bounds__(kFsThreads) fine_step_kernel(const BoxDesc* __restrict__ boxes, int box0,
                                                                  int parity) {
  using TP = typename PR::TP;
  using RA = TP;  // arithmetic: FP64 for FP64 storage, FP32 otherwise
  __shared__ RA sP[kFsPN];
  __shared__ RA sG[3][kFsGN];
  __shared__ RA sU[3][kFsUN];
  const BoxDesc& b = boxes[box0 + blockIdx.y];
  const int nx = b.nx, ny = b.ny;
  const int fx = 2 * nx, fy = 2 * ny, fz = 2 * b.nz;
  const int ntx = (fx + kFsTX - 1) / kFsTX, nty = (fy + kFsTY - 1) / kFsTY;
  const int tiles = ntx * nty * ((fz + kHoZ - 1) / kHoZ);
  const int64_t n = static_cast<int64_t>(nx) * ny * b.nz;
  const int64_t cplane = static_cast<int64_t>(nx) * ny;
  const int64_t fplane = static_cast<int64_t>(fx) * fy;
  const gptr<const TP> fphi = (gptr<const TP>)b.fphi[parity];
  const gptr<TP> fout = (gptr<TP>)b.fphi[1 - parity];
  const TP* __restrict__ u = static_cast<const TP*>(b.aux);
  const RA kac = static_cast<RA>(b.kappa_ac), mob = static_cast<RA>(b.mobility);
  constexpr RA kInvH = 2, kInvH2 = 4;  // 1 / h, 1 / h^2
  const int tid = threadIdx.x;
  // this thread's flux column in the region (threads past kFsGN take column
  // 0 for their reads and store no flux) and whether it is an output column
  const bool gthread = tid < kFsGN;
  const int gx = gthread ? tid % kFsGX : 0, gy = gthread ? tid / kFsGX : 0;
  const bool inner = gthread && gx >= 1 && gx <= kFsTX && gy >= 1 && gy <= kFsTY;
  constexpr int kPer = (kFsPN + kFsThreads - 1) / kFsThreads;
  constexpr int kPerU = (3 * kFsUN + kFsThreads - 1) / kFsThreads;
  for (int t = blockIdx.x; t < tiles; t += gridDim.x) {  // uniform over the workgroup
    const int x0 = (t % ntx) * kFsTX, y0 = ((t / ntx) % nty) * kFsTY, z0 = (t / (ntx * nty)) * kHoZ;
    const int z1 = min(z0 + kHoZ, fz);
    const int X = x0 - 1 + gx, Y = y0 - 1 + gy;  // unmapped fine column of the flux
    const bool active = inner && X < fx && Y < fy;
    // phi staging: this thread's elements, mapped columns (far columns clamp)
    int64_t ecol[kPer];
    for (int j = 0; j < kPer; ++j) {
      const int e = min(tid + kFsThreads * j, kFsPN - 1);
      const int xe = x0 - 2 + e % kFsPX, ye = y0 - 2 + e / kFsPX;
      ecol[j] = fine_at(b, map_axis(xe, fx, b.wall[0]), map_axis(ye, fy, b.wall[1]), 0);
    }
    // staged values of a plane in registers: two buffers, the even and the
    // odd planes of the march, each loaded two planes before it is staged
    TP bufA[kPer], bufB[kPer];
    auto load = [&](int r, TP* buf) {  // unmapped fine plane r, continued
      const int64_t zoff = map_axis(r, fz, b.wall[2]) * fplane;
      for (int j = 0; j < kPer; ++j) buf[j] = fphi[ecol[j] + zoff];
    };
    auto commit = [&](const TP* buf) {
      for (int j = 0; j < kPer; ++j)
        if (tid + kFsThreads * j < kFsPN) sP[tid + kFsThreads * j] = dec<RA>(buf[j], 0.f, 1.f);
    };
    // velocity staging: coarse columns [cx0, cx0 + kFsUX) x [cy0, cy0 + kFsUY),
    // this thread's elements, their physical columns and the signs of the odd
    // continuation in x and y
    const int cx0 = ((x0 - 1) >> 1) - 1, cy0 = ((y0 - 1) >> 1) - 1;
    int64_t ucol[kPerU];
    bool uneg[kPerU];
    for (int j = 0; j < kPerU; ++j) {
      const int e = min(tid + kFsThreads * j, 3 * kFsUN - 1);
      const int a = e / kFsUN, r = e % kFsUN;
      int kx, ky;
      const int cx = map_axis(cx0 + r % kFsUX, nx, b.wall[0], kx);
      const int cy = map_axis(cy0 + r / kFsUX, ny, b.wall[1], ky);
      ucol[j] = a * n + static_cast<int64_t>(cy) * nx + cx;
      uneg[j] = ((kx + ky) & 1) != 0;
    }
    RA unext[kPerU];
    auto load_u = [&](int p) {  // unmapped coarse plane p
      int kz;
      const int64_t zoff = map_axis(p, b.nz, b.wall[2], kz) * cplane;
      for (int j = 0; j < kPerU; ++j) {
        const RA v = static_cast<RA>(u[ucol[j] + zoff]);
        unext[j] = (uneg[j] != (kz != 0)) ? -v : v;
      }
    };
    auto commit_u = [&]() {
      for (int j = 0; j < kPerU; ++j) {
        const int e = tid + kFsThreads * j;
        if (e < 3 * kFsUN) sU[e / kFsUN][e % kFsUN] = unext[j];
      }
    };
    // the flux column's coarse cell X >> 1 (weight 3/4) and its neighbour
    // towards the fine node (weight 1/4), as staged columns
    const int li = (X >> 1) - cx0, lj = (Y >> 1) - cy0;
    const int lni = li + ((X & 1) ? 1 : -1), lnj = lj + ((Y & 1) ? 1 : -1);
    auto bilinear = [&](RA B[3]) {
      for (int a = 0; a < 3; ++a)
        B[a] = RA(0.75) * (RA(0.75) * sU[a][lj * kFsUX + li] + RA(0.25) * sU[a][lj * kFsUX + lni]) +
               RA(0.25) * (RA(0.75) * sU[a][lnj * kFsUX + li] + RA(0.25) * sU[a][lnj * kFsUX + lni]);
    };
    // filtered values of the staged phi plane at the flux column:
    // F[0] = s_x s_y phi, F[1] = s_y d_x phi, F[2] = s_x d_y phi, F[3] = phi,
    // s = (1, 4, 1), d = (-1, 0, 1)
    auto filt = [&](RA F[4]) {
      const int c0 = (gy + 1) * kFsPX + gx + 1;
      RA sx[3], dx[3];
      for (int cy = 0; cy < 3; ++cy) {
        const int e = c0 + (cy - 1) * kFsPX;
        const RA l = sP[e - 1], c = sP[e], h = sP[e + 1];
        sx[cy] = l + RA(4) * c + h;
        dx[cy] = h - l;
      }
      F[0] = sx[0] + RA(4) * sx[1] + sx[2];
      F[1] = dx[0] + RA(4) * dx[1] + dx[2];
      F[2] = sx[2] - sx[0];
      F[3] = sP[c0];
    };
    // filtered values of the flux plane at the output column:
    // v[0] = sum w cx Gx, v[1] = sum w cy Gy, v[2] = sum w Gz, w = (1, 4, 1) x (1, 4, 1)
    auto filt_g = [&](RA v[3]) {
      const int c0 = gy * kFsGX + gx;
      RA hx = 0, hy = 0, hz = 0;
      for (int cy = -1; cy <= 1; ++cy)
        for (int cx = -1; cx <= 1; ++cx) {
          const RA w = (cx ? RA(1) : RA(4)) * (cy ? RA(1) : RA(4));
          const int e = c0 + cy * kFsGX + cx;
          if (cx) hx += w * RA(cx) * sG[0][e];
          if (cy) hy += w * RA(cy) * sG[1][e];
          hz += w * sG[2][e];
        }
      v[0] = hx;
      v[1] = hy;
      v[2] = hz;
    };
    // bilinear sums of the coarse planes around the first flux plane
    // (unmapped fine plane z0 - 1, coarse plane (z0 - 1) >> 1)
    RA Bm[3], B0[3], Bp[3];
    {
      const int c0 = (z0 - 1) >> 1;
      auto first = [&](int p, RA B[3]) {
        load_u(p);
        commit_u();
        __syncthreads();
        bilinear(B);
        __syncthreads();
      };
      first(c0 - 1, Bm);
      first(c0, B0);
      first(c0 + 1, Bp);
    }
    bool u_pending = false;
    RA F[4][4] = {}, V[3][3] = {};
    // one staged plane r: its values come from buf, which then takes plane
    // r + 2 (in flight while this plane and the next are filtered and used)
    auto plane = [&](int r, TP* buf) {
      commit(buf);
      if (u_pending) commit_u();
      __syncthreads();
      if (r + 2 <= z1 + 1) load(r + 2, buf);
      for (int k = 0; k < 4; ++k) {
        F[0][k] = F[1][k];
        F[1][k] = F[2][k];
        F[2][k] = F[3][k];
      }
      filt(F[3]);
      RA Bnew[3];
      const bool fresh = u_pending;
      if (fresh) bilinear(Bnew);
      u_pending = false;
      if (r >= z0) {  // flux plane p = r - 1 from the filtered planes r - 2 .. r
        const int p = r - 1, c = p >> 1;
        if (fresh) {  // c advanced: planes c - 1, c, c + 1
          for (int a = 0; a < 3; ++a) {
            Bm[a] = B0[a];
            B0[a] = Bp[a];
            Bp[a] = Bnew[a];
          }
        }
        if ((p & 1) && p + 1 <= z1) {  // the next flux plane starts coarse plane c + 1
          load_u(c + 2);
          u_pending = true;
        }
        const bool odd = (p & 1) != 0;
        const RA phi = F[2][3];
        const RA g[3] = {(F[1][1] + RA(4) * F[2][1] + F[3][1]) * (kInvH / RA(72)),
                         (F[1][2] + RA(4) * F[2][2] + F[3][2]) * (kInvH / RA(72)),
                         (F[3][0] - F[1][0]) * (kInvH / RA(72))};
        const RA inv = rcp_newton(sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + RA(1e-12));
        const RA pp = phi * (RA(1) - phi);
        if (gthread)
          for (int a = 0; a < 3; ++a) {
            const RA uf = RA(0.75) * B0[a] + RA(0.25) * (odd ? Bp[a] : Bm[a]);
            sG[a][tid] = phi * uf + kac * (pp * g[a] * inv);
          }
      }
      __syncthreads();
      if (r < z0) return;
      for (int k = 0; k < 3; ++k) {
        V[0][k] = V[1][k];
        V[1][k] = V[2][k];
      }
      if (inner) filt_g(V[2]);
      if (r < z0 + 2 || !active) return;  // output plane r - 2 needs flux planes r - 3 .. r - 1
      const int z = r - 2;
      const RA phi = F[1][3];
      const RA div = ((V[0][0] + RA(4) * V[1][0] + V[2][0]) + (V[0][1] + RA(4) * V[1][1] + V[2][1]) +
                      (V[2][2] - V[0][2])) * (kInvH / RA(72));
      const RA lap = ((F[0][0] + RA(4) * F[1][0] + F[2][0]) * RA(1.0 / 36.0) - RA(6) * phi) * kInvH2;
      fout[fine_at(b, X, Y, z)] = Enc<TP>::go(phi - div + mob * lap, 0.f, 1.f);
    };
    // staged planes z0 - 2 .. z1 + 1 (at least 4), two per trip
    load(z0 - 2, bufA);
    load(z0 - 1, bufB);
    for (int r = z0 - 2; r <= z1 + 1; r += 2) {
      plane(r, bufA);
      if (r + 1 <= z1 + 1) plane(r + 1, bufB);
    }
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
  int64_t nb = (max_nodes + 256 * 16 - 1) / (256 * 16);
  return static_cast<int>(nb < 1 ? 1 : (nb > 4096 ? 4096 : nb));
}

int high_order_phase_tiles(int nx, int ny, int nz) {
  return ((nx + kHoTX - 1) / kHoTX) * ((ny + kHoTY - 1) / kHoTY) * ((nz + kHoZ - 1) / kHoZ);
}

hipError_t launch_high_order_phase(int precision, bool gc, bool literal, const BoxDesc* d_boxes, int box0, int nbox,
                                   int parity, int flux_blocks, int phase_tiles, hipStream_t stream) {
  if (nbox <= 0 || flux_blocks <= 0 || phase_tiles <= 0) return hipErrorInvalidValue;
  return dispatch(precision, [&](auto pr) {
    using PR = decltype(pr);
    if (gc)
      hipLaunchKernelGGL((ho_flux_kernel<PR, true, true>), dim3(flux_blocks, nbox), dim3(256), 0, stream, d_boxes, box0, parity);
    else
      hipLaunchKernelGGL((ho_flux_kernel<PR, false, true>), dim3(flux_blocks, nbox), dim3(256), 0, stream, d_boxes, box0,
                         parity);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (literal)
      hipLaunchKernelGGL((ho_phase_kernel<PR, true>), dim3(phase_tiles, nbox), dim3(256), 0, stream, d_boxes, box0,
                         parity);
    else
      hipLaunchKernelGGL((ho_phase_kernel<PR, false>), dim3(phase_tiles, nbox), dim3(256), 0, stream, d_boxes, box0,
                         parity);
    return hipGetLastError();
  });
}

hipError_t launch_fine_init(int precision, const BoxDesc& box, const BoxDesc* d_box, int parity, hipStream_t stream) {
  const int64_t nf = 8 * static_cast<int64_t>(box.nx) * box.ny * box.nz;
  const int64_t n = nf / 8;
  return dispatch(precision, [&](auto pr) {
    using PR = decltype(pr);
    hipLaunchKernelGGL((fine_prolong_kernel<PR>), dim3(grid_for(nf, 256)), dim3(256), 0, stream, box, parity);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((fine_restrict_kernel<PR>), dim3(grid_for(n, 256), 1), dim3(256), 0, stream, d_box, 0, parity);
    return hipGetLastError();
  });
}

hipError_t launch_fine_set(int precision, const BoxDesc& box, const BoxDesc* d_box, int parity, const double* d_src,
                           hipStream_t stream) {
  const int64_t nf = 8 * static_cast<int64_t>(box.nx) * box.ny * box.nz;
  const int64_t n = nf / 8;
  return dispatch(precision, [&](auto pr) {
    using PR = decltype(pr);
    hipLaunchKernelGGL((fine_encode_kernel<PR>), dim3(grid_for(nf, 256)), dim3(256), 0, stream, box, parity, d_src, nf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((fine_restrict_kernel<PR>), dim3(grid_for(n, 256), 1), dim3(256), 0, stream, d_box, 0, parity);
    return hipGetLastError();
  });
}

hipError_t launch_fine_get(int precision, const BoxDesc& box, int parity, double* d_dst, hipStream_t stream) {
  const int64_t nf = 8 * static_cast<int64_t>(box.nx) * box.ny * box.nz;
  return dispatch(precision, [&](auto pr) {
    using PR = decltype(pr);
    hipLaunchKernelGGL((fine_decode_kernel<PR>), dim3(grid_for(nf, 256)), dim3(256), 0, stream, box, parity, d_dst, nf);
    return hipGetLastError();
  });
}

hipError_t launch_fine_gather(int precision, const BoxDesc& box, int parity, const int64_t* d_idx, int64_t n,
                              double* d_out, hipStream_t stream) {
  return dispatch(precision, [&](auto pr) {
    using PR = decltype(pr);
    hipLaunchKernelGGL((fine_gather_kernel<PR>), dim3(grid_for(n, 256)), dim3(256), 0, stream, box, parity, d_idx, n,
                       d_out);
    return hipGetLastError();
  });
}

int fine_tiles(int nx, int ny, int nz) { return fine_step_tiles(nx, ny, nz); }

hipError_t launch_fine_phase(int precision, bool gc, const BoxDesc* d_boxes, int box0, int nbox, int parity,
                             int u_blocks, int step_tiles, int restrict_blocks, hipStream_t stream) {
  if (nbox <= 0 || u_blocks <= 0 || step_tiles <= 0 || restrict_blocks <= 0) return hipErrorInvalidValue;
  return dispatch(precision, [&](auto pr) {
    using PR = decltype(pr);
    if (gc)
      hipLaunchKernelGGL((ho_flux_kernel<PR, true, false>), dim3(u_blocks, nbox), dim3(256), 0, stream, d_boxes, box0,
                         parity);
    else
      hipLaunchKernelGGL((ho_flux_kernel<PR, false, false>), dim3(u_blocks, nbox), dim3(256), 0, stream, d_boxes, box0,
                         parity);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((fine_step_kernel<PR>), dim3(step_tiles, nbox), dim3(kFsThreads), 0, stream, d_boxes, box0,
                       parity);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((fine_restrict_kernel<PR>), dim3(restrict_blocks, nbox), dim3(256), 0, stream, d_boxes, box0,
                       1 - parity);
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
