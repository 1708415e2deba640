// State layout shared by the device code and the host runtime of liblbm.so:
// the per-box descriptor the kernels read and the work items of the fused
// step.  Not part of the public ABI.
#pragma once

#include <cstdint>

namespace lbm {

constexpr int kFields = 11;  // phi, P, Jx, Jy, Jz, Qxx, Qyy, Qzz, Qxy, Qxz, Qyz

// Per-box constants and state pointers, resident in device memory; read with
// uniform (scalar) loads by every workgroup working on the box.
struct BoxDesc {
  // ping-pong state buffers, index = parity:
  //   phi[s]: [nz][ny][pitch] phase field (storage type of phi)
  //   mom[s]: [nz][nmom][ny][pitch] moments P, Jx, Jy, Jz, Qxx, Qyy, Qzz, Qxy, Qxz, Qyz
  //           (each z plane holds its nmom moment planes back to back;
  //           nmom = 4, P and J only, for the gradient closure)
  void* phi[2];
  void* mom[2];
  int32_t nx, ny, nz;
  int32_t wall[3];        // 1 if the axis has walls
  int32_t flags;          // LBM_LITERAL_ADVECTION | LBM_GRADIENT_CLOSURE | LBM_HIGH_ORDER_AC
  int32_t nmom;           // moment fields stored per node: 10, or 4 (gradient closure)
  double rho_g, drho;     // rho = rho_g + phi * drho
  double nu_g, dnu;       // nu = nu_g + phi * dnu
  double beta4;           // 4 beta = 48 sigma / W
  double kappa_mu;        // 3 sigma W / 2
  double mobility;        // M
  double kappa_ac;        // 4 M / W
  double grav[3];
  double rho_ref;
  float enc_off[10];      // moment k stored as (v - off) * scale in 16-bit modes
  float enc_scale[10];
  float enc_inv[10];      // 1 / scale (exact: powers of two)
  int32_t whole_rows;     // 1 if every stored row starts on a 64-byte boundary
                          // (buffer bases multiples of 64 bytes)
  int32_t zero_offsets;   // 1 if every enc_off is +0 (the default encoding)
  int32_t pitch;          // elements from one stored row to the next (>= nx; the
                          // padding after column nx-1 is never read or written)
  void* aux;              // LBM_HIGH_ORDER_AC: 6 compact planes of nx*ny*nz values
                          // of the phi storage type (u, then phi (1 - phi) n4)
                          // of the step's level n; LBM_FINE_PHASE: 3 such
                          // planes (u); else NULL
  // LBM_FINE_PHASE: the phase field on the grid refined by 2 per axis,
  // [2nz][2ny][2nx] (compact) of the phi storage type, per parity; NULL
  // otherwise.
  void* fphi[2];
};

// One unit of work of the fused step: an output tile (x0, y0) of one box,
// marched over output planes [z0, z1).
struct Item {
  int32_t box, x0, y0, z0, z1, pad[3];
};

enum Precision { kF64 = 0, kF32 = 1, kF16 = 2, kBF16 = 3 };

}  // namespace lbm
