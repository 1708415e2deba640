// Device code of liblbm.so for gfx950 (MI355X).
//
// fused_step: one time step of the thread-safe D3Q27 lattice Boltzmann
// solver with the conservative Allen-Cahn phase field (arXiv 2501.00846,
// Sec. II.D), as a single pull-style kernel that reads the 11 moment fields of
// buffer s and writes those of buffer 1 - s; every thread writes only its own
// node, so no two threads ever touch the same output (the thread-safe
// property of Sec. II.B).
//
// Work decomposition.  A workgroup owns an output tile of (BX-2) x (BY-2)
// columns of one box and marches it along z over planes [z0, z1).  Its BX x BY
// threads map one-to-one onto the tile plus a one-column halo ring.  For every
// node plane p the workgroup
//   (A) stages phi of plane p+1 with a two-column halo in LDS and filters it
//       in x-y (per-axis stencils (1,4,1) and (-1,0,1)); with the filtered
//       planes p-1, p, p+1 held in registers each thread gets the isotropic
//       gradient and Laplacian of Sec. II.C at its node of plane p;
//   (B) computes at that node rho, nu, omega, mu, the forces of Sec.
//       II.C, the acceleration a = F/rho, u = J + a/2, the regularisation
//       tensor a2 = Q + a a/4 (Eq. hermite_neq2 with the shifted equilibrium),
//       the 17 monomial coefficients of the post-collision populations
//       f_post(c) = w(c) g(c) (Eqs. eqts, noneqts, guoforce, LBexp), their 27
//       values by sum factorisation, and the phase-field flux
//       G = phi u + (4M/W) phi (1 - phi) n;
//   (C) exchanges f_post and G through LDS: each interior thread pulls the
//       populations that stream into its column from the 3 x 3 neighbour
//       columns and adds their moments to the running sums of output planes
//       p-1, p, p+1 (registers), and likewise the divergence of G.  Output
//       plane p-1 is then complete: Q' = Pi - cs^2 P' I - J' J', the FTCS
//       phase update phi' = phi + M lap(phi) - div(G), and 11 stores (5
//       with the gradient closure, see fused_step).
// Halo work is recomputed by the halo-ring threads; nothing but the 11 state
// fields goes to or comes from HBM.
//
// Walls (no-slip, neutral wetting): half-way bounce-back f_i(x) =
// f_post_opp(i)(x) when x - c_i is behind a wall; phi ghosts mirror the
// interior; ghost flux G = phi (-u) + kappa_AC phi (1-phi) n with the normal
// from the mirrored phi (reflected component).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device_common.h"
#include "lbm_internal.h"

namespace lbm {
namespace {

// A wave-uniform address, pinned to scalar registers and opaque to the
// optimiser, so that a load or store at base + 32-bit lane offset is issued in
// the scalar-base form (no per-lane 64-bit address arithmetic) instead of being
// strength-reduced into per-lane pointer increments.
template <class T>
__device__ __forceinline__ gptr<T> sbase(gptr<T> p) {
  uint64_t a = reinterpret_cast<uint64_t>(p);
  asm("" : "+s"(a));
  return reinterpret_cast<gptr<T>>(a);
}

// A per-lane 32-bit byte offset, re-materialised where it is used so that its
// zero extension is visible next to the access (instruction selection matches
// the scalar-base form only within one basic block).
__device__ __forceinline__ uint32_t lane_off(uint32_t v) {
  asm("" : "+v"(v));
  return v;
}

// Store of a freshly computed output element, with the non-temporal hint when
// NT is set: the next step reads the element back only after the whole state
// has streamed through the caches, and the hint keeps it from displacing the
// halo lines that neighbouring tiles re-read.  The hint pays only where a
// wave's stores cover whole 64-byte segments; on partly covered segments
// non-temporal writes are several times slower, so the kernel uses it only
// for 4- and 8-byte storage, tiles whose lanes store whole aligned rows, and
// boxes whose rows start on 64-byte boundaries.
template <bool NT, class T>
__device__ __forceinline__ void store_out(gptr<T> p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Plane index map for a uniform q in [-2, n+1]: fast path inside the domain.
__device__ __forceinline__ int map_plane(int q, int n, int wall) {
  if (q >= 0 && q < n) return q;
  return map_axis(q, n, wall);
}

// LDS slot of the population with direction (cx, cy, cz), (cx, cy) != (0, 0).
__host__ __device__ constexpr int fslot(int cx, int cy, int cz) {
  return (((cy + 1) * 3 + (cx + 1)) - ((((cy + 1) * 3 + (cx + 1)) > 4) ? 1 : 0)) * 3 + (cz + 1);
}

// x-y parts of the isotropic divergence of a flux stored per tile position:
// hx = sum_cy w(cy) (G_x(+1, cy) - G_x(-1, cy)), hy likewise along y, and
// hz = sum w(cx) w(cy) G_z(cx, cy), weights w = (1, 4, 1); each sum starts from
// its first term.
template <class R, class F>
__device__ __forceinline__ void div_sums(const F& G, R& hx, R& hy, R& hz) {
  hx = G(0, 1, -1) - G(0, -1, -1);
  hx += R(4) * (G(0, 1, 0) - G(0, -1, 0));
  hx += G(0, 1, 1) - G(0, -1, 1);
  hy = G(1, -1, 1) - G(1, -1, -1);
  hy += R(4) * (G(1, 0, 1) - G(1, 0, -1));
  hy += G(1, 1, 1) - G(1, 1, -1);
  hz = G(2, -1, -1);
#pragma unroll
  for (int k = 1; k < 9; ++k) {
    const int cx = k % 3 - 1, cy = k / 3 - 1;
    const R w = (cx == 0 ? R(4) : R(1)) * (cy == 0 ? R(4) : R(1));
    hz += w * G(2, cx, cy);
  }
}

// Moment accumulator of one output plane: P, J (3), Pi = sum f c c (6).
template <class R> struct Acc {
  R p, jx, jy, jz, xx, yy, zz, xy, xz, yz;
  __device__ void zero() { p = jx = jy = jz = xx = yy = zz = xy = xz = yz = R(0); }
};

// Add the moments of 9 populations sharing c_z = cz, each weighted by its
// lattice weight: v[(cy+1)*3 + (cx+1)] holds g(c)/216 and the population is
// w1(cx) w1(cy) w1(cz) v with w1 = (1, 4, 1) (216 w(c)).
// FRESH: the accumulator holds nothing yet, so the sums are assigned (adding
// them to zero would cost an instruction each: x + 0 is not x for x = -0).
template <class R, int CZ, bool FRESH = false>
__device__ __forceinline__ void accum_group(const R* v, Acc<R>& a) {
  // along x for each c_y row: s0 = sum w1 v, s1 = sum cx w1 v, s2 = sum cx^2 w1 v
  R s0[3], s1[3], s2[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const R l = v[r * 3 + 0], c = v[r * 3 + 1], h = v[r * 3 + 2];
    s2[r] = h + l;
    s1[r] = h - l;
    s0[r] = s2[r] + R(4) * c;
  }
  const R m02 = s0[2] + s0[0];
  const R m00 = m02 + R(4) * s0[1];
  const R m01 = s0[2] - s0[0];
  const R m10 = s1[0] + s1[2] + R(4) * s1[1];
  const R m11 = s1[2] - s1[0];
  const R m20 = s2[0] + s2[2] + R(4) * s2[1];
  if constexpr (FRESH) {
    static_assert(CZ > 0, "only the group entering a new output plane starts it");
    a.p = m00;
    a.jx = m10;
    a.jy = m01;
    a.xx = m20;
    a.yy = m02;
    a.xy = m11;
    a.zz = m00;
    a.jz = m00;
    a.xz = m10;
    a.yz = m01;
    return;
  }
  if (CZ == 0) {
    a.p += R(4) * m00;
    a.jx += R(4) * m10;
    a.jy += R(4) * m01;
    a.xx += R(4) * m20;
    a.yy += R(4) * m02;
    a.xy += R(4) * m11;
    return;
  }
  a.p += m00;
  a.jx += m10;
  a.jy += m01;
  a.xx += m20;
  a.yy += m02;
  a.xy += m11;
  {
    a.zz += m00;
    if (CZ > 0) { a.jz += m00; a.xz += m10; a.yz += m01; }
    else        { a.jz -= m00; a.xz -= m10; a.yz -= m01; }
  }
}

// Lane -> tile position (tx, ty).  When the output rows are a multiple of 32
// columns wide, the (BX-2) x (BY-2) output columns come first, row by row:
// every wavefront then covers whole, aligned output rows, so its loads and
// stores of a field are full memory segments (each partial segment costs the
// vector L1 a request of its own, and stores are limited by those requests).
// The halo ring follows: top row, bottom row, left column, right column.
// Other shapes keep the row-major order of the block.
template <int BX, int BY>
__device__ __forceinline__ void lane_position(int tid, int& tx, int& ty) {
  constexpr int IX = BX - 2, IY = BY - 2, NI = IX * IY;
  if constexpr (IX % 32 != 0) {
    tx = tid % BX;
    ty = tid / BX;
    return;
  }
  if (tid < NI) {
    ty = tid / IX + 1;
    tx = tid % IX + 1;
    return;
  }
  int h = tid - NI;
  if (h < BX) { tx = h; ty = 0; return; }
  h -= BX;
  if (h < BX) { tx = h; ty = BY - 1; return; }
  h -= BX;
  if (h < IY) { tx = 0; ty = h + 1; return; }
  h -= IY;
  tx = BX - 1;
  ty = h + 1;
}

template <int BX, int BY, class PR, bool GC>
struct FusedShared {
  using R = typename PR::R;
  static constexpr int NT = BX * BY;
  static constexpr int NP = (BY + 2) * (BX + 2);
  R phi[NP];
  R jp[GC ? 3 * NP : 1];  // gradient closure: J of the staged plane, halo 2
  R f[24 * NT];
  R g[3 * NT];
  R gg[3 * NT];
};

// 16-bit storage keeps the moments in pairs: one 32-bit word per node holds
// fields 2p (low half) and 2p + 1 (high half) of pair plane p, so that a step
// issues half as many moment loads and stores (a wave's store costs the
// vector memory path about the same for 2- and 4-byte elements).
template <class TM>
__device__ __forceinline__ TM half_of(uint32_t w, int hi) {
  return __builtin_bit_cast(TM, static_cast<uint16_t>(hi ? (w >> 16) : w));
}
// Encodes moments v0 (low half) and v1 (high half) into one word; both are
// rounded by one packed conversion (v_cvt_pk_f16_f32 / v_cvt_pk_bf16_f32).
// ZO: both offsets are +0, whose subtraction changes no value.
template <class TM, bool ZO>
__device__ __forceinline__ uint32_t encode_pair(float v0, float v1, float o0, float s0, float o1, float s1) {
  if constexpr (ZO) {
    o0 = 0.f;  // (v - (+0)) * s == v * s, bitwise (-0 - +0 = -0)
    o1 = 0.f;
  }
  if constexpr (std::is_same_v<TM, _Float16>) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 h = {Enc<TM>::go(v0, o0, s0), Enc<TM>::go(v1, o1, s1)};
    return __builtin_bit_cast(uint32_t, h);
  } else {
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    const f2 f = {(v0 - o0) * s0, (v1 - o1) * s1};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, b2));
  }
}

// ---------------------------------------------------------------------------
// The fused step
// ---------------------------------------------------------------------------
// Occupancy targets: FP64 needs 210-256 VGPRs (2 waves per SIMD); the FP32
// arithmetic instantiations are held to 128 VGPRs for 4 waves per SIMD (the
// moment closure fits; the gradient closure spills a few registers).
template <class PR> struct WavesPerEU { static constexpr int v = 4; };
template <> struct WavesPerEU<PF64> { static constexpr int v = 2; };

// GC selects the gradient-closure variant: the state holds phi, P and J only
// (4 moment fields per plane instead of 10) and a2 is rebuilt from the
// isotropic gradient of J, a2 = -(cs^2/omega)(grad J + grad J^T) (the
// velocity-gradient a2 given with Eq. noneqts), which also feeds the viscous
// correction.  J is staged like phi (two-column halo) so that the halo-ring
// nodes get their gradient too; its ghost values are minus the mirrored ones
// (sign (-1)^(walls crossed)), the ghost rule of the velocity.
template <int BX, int BY, class PR, bool GC>
__global__ void __launch_bounds__(BX * BY) __attribute__((amdgpu_waves_per_eu(WavesPerEU<PR>::v)))
fused_step(const BoxDesc* __restrict__ boxes, const Item* __restrict__ items, int n_items,
           int parity) {
  using TM = typename PR::TM;
  using TP = typename PR::TP;
  using R = typename PR::R;
  constexpr int NT = BX * BY;
  constexpr int PX = BX + 2;
  constexpr int PY = BY + 2;
  constexpr int NM = GC ? 4 : 10;  // moment fields per plane
  constexpr int NL = GC ? 1 : 10;  // of them loaded per lane (the closure takes J from its LDS patch)
  constexpr bool PAIR = sizeof(TM) == 2;  // 16-bit moments stored in pairs (32-bit words)
  // non-temporal output stores possible: 4- or 8-byte stored words and the
  // interior-first lane map (32 output columns per row)
  constexpr bool NTS = (sizeof(TM) >= 4 || PAIR) && (BX - 2) % 32 == 0;
  __shared__ FusedShared<BX, BY, PR, GC> sh;

  const int tid = threadIdx.x;
  int tx, ty;
  lane_position<BX, BY>(tid, tx, ty);
  const int sp = ty * BX + tx;  // LDS slot of this thread's tile position

  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const Item item = items[it];
    const BoxDesc& b = boxes[item.box];
    const int nx = b.nx, ny = b.ny, nz = b.nz;
    const int wx = b.wall[0], wy = b.wall[1], wz = b.wall[2];
    const int pitch = b.pitch;
    const int64_t plane = static_cast<int64_t>(pitch) * ny;

    const int x = item.x0 - 1 + tx;
    const int y = item.y0 - 1 + ty;
    int crx, cry;
    const int xm = map_axis(x, nx, wx, crx);
    const int ym = map_axis(y, ny, wy, cry);
    const int64_t col = static_cast<int64_t>(ym) * pitch + xm;
    const bool out_col = tx >= 1 && tx <= BX - 2 && ty >= 1 && ty <= BY - 2 && x < nx && y < ny;
    // per-lane flags kept in one VGPR; decoded where used inside the z loop
    // (bit 0/1: ghost column mirrored in x/y; bits 2-5: output node next to
    // the low-x / high-x / low-y / high-y wall)
    const uint32_t lflags0 = (crx ? 1u : 0u) | (cry ? 2u : 0u) |
                             ((wx && x == 0) ? 4u : 0u) | ((wx && x == nx - 1) ? 8u : 0u) |
                             ((wy && y == 0) ? 16u : 0u) | ((wy && y == ny - 1) ? 32u : 0u);

    // uniform: does this tile touch a wall in x or y?
    const bool wall_tile = (wx && (item.x0 == 0 || item.x0 + BX - 2 >= nx)) ||
                           (wy && (item.y0 == 0 || item.y0 + BY - 2 >= ny));

    // state views: phi [z][y][x]; moments [z][k][y][x] (plane-interleaved;
    // in 16-bit storage [z][k/2][y][x] of 32-bit pairs)
    const gptr<const TP> s_phi_g = (gptr<const TP>)(b.phi[parity]);
    const gptr<const TM> s_mom = (gptr<const TM>)(b.mom[parity]);
    const gptr<TP> d_phi_g = (gptr<TP>)(b.phi[1 - parity]);
    const gptr<TM> d_mom = (gptr<TM>)(b.mom[1 - parity]);
    const uint32_t ucol = static_cast<uint32_t>(col);
    const uint32_t voff_p = ucol * static_cast<uint32_t>(sizeof(TP));  // byte offset in a phi plane
    const uint32_t voff_m = ucol * static_cast<uint32_t>(sizeof(TM));  // byte offset in a moment plane
    const uint32_t voff_w = ucol * 4u;  // byte offset in a pair plane (16-bit storage)
    const int64_t plane_bp = plane * static_cast<int64_t>(sizeof(TP));
    const int64_t plane_bm = plane * static_cast<int64_t>(sizeof(TM));

    const R beta4 = static_cast<R>(b.beta4);
    const R kappa_mu = static_cast<R>(b.kappa_mu);
    const R kappa_ac = static_cast<R>(b.kappa_ac);
    const R mob = static_cast<R>(b.mobility);
    const R drho3 = static_cast<R>(b.drho * (1.0 / 3.0));
    const R grx = static_cast<R>(b.grav[0]), gry = static_cast<R>(b.grav[1]), grz = static_cast<R>(b.grav[2]);
    const bool literal = (b.flags & 1) != 0;

    const int z0 = item.z0, z1 = item.z1;
    const int p_first = (wz && z0 == 0) ? 0 : z0 - 1;
    const int p_last = (wz && z1 == nz) ? nz - 1 : z1;

    // --- stage phi of plane q into LDS (halo columns resolved once per tile)
    constexpr int NPH = (PX * PY + NT - 1) / NT;
    uint32_t phcol[NPH];
#pragma unroll
    for (int j = 0; j < NPH; ++j) {
      const int e = tid + j * NT;
      const int i = e % PX, jj = e / PX;
      phcol[j] = static_cast<uint32_t>(map_axis(item.y0 - 2 + jj, ny, wy) * pitch + map_axis(item.x0 - 2 + i, nx, wx)) *
                 static_cast<uint32_t>(sizeof(TP));
    }
    // gradient closure: bit j set when halo element j lies across an odd
    // number of x/y walls (its J enters with the opposite sign)
    uint32_t jflip = 0;
    if constexpr (GC) {
#pragma unroll
      for (int j = 0; j < NPH; ++j) {
        const int e = tid + j * NT;
        const int i = e % PX, jj = e / PX;
        int cx, cy;
        (void)map_axis(item.x0 - 2 + i, nx, wx, cx);
        (void)map_axis(item.y0 - 2 + jj, ny, wy, cy);
        jflip |= static_cast<uint32_t>(cx ^ cy) << j;
      }
    }
    // phi of one plane at this thread's halo elements: loaded one plane ahead
    // into registers, stored to LDS when the plane is needed.  Addresses are a
    // uniform plane base plus a 32-bit per-lane byte offset (a plane holds at
    // most 2^28 nodes, so offsets within it fit), which keeps the per-load
    // address arithmetic off the vector ALUs.
    auto load_phi = [&](int q, R* v) {
      const gptr<const char> src = sbase((gptr<const char>)s_phi_g + static_cast<int64_t>(map_plane(q, nz, wz)) * plane_bp);
#pragma unroll
      for (int j = 0; j < NPH; ++j) v[j] = static_cast<R>(*(gptr<const TP>)(src + lane_off(phcol[j])));
    };
    auto store_phi = [&](const R* v) {
#pragma unroll
      for (int j = 0; j < NPH; ++j) {
        const int e = tid + j * NT;
        if (j < NPH - 1 || e < PX * PY) sh.phi[e] = v[j];
      }
    };
    // returns (A', Bx', By', phi_c): A' = s_x s_y phi, Bx' = s_y d_x phi,
    // By' = s_x d_y phi with s = (1,4,1), d = (-1,0,1)
    auto filter_phi = [&](R* F) {
      R dx[3], sx[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const R* row = &sh.phi[(ty + r) * PX + tx];
        const R l = row[0], c = row[1], h = row[2];
        dx[r] = h - l;
        sx[r] = l + R(4) * c + h;
        if (r == 1) F[3] = c;
      }
      F[0] = sx[0] + R(4) * sx[1] + sx[2];
      F[1] = dx[0] + R(4) * dx[1] + dx[2];
      F[2] = sx[2] - sx[0];
    };

    // gradient closure: J (fields 1-3) at the same halo elements as phi
    constexpr int NP = PX * PY;
    auto load_J = [&](int q, R (*v)[NPH]) {
      const gptr<const char> base = (gptr<const char>)s_mom + static_cast<int64_t>(map_plane(q, nz, wz)) * NM * plane_bm;
      if constexpr (PAIR) {
        // Jx: high half of pair 0 (P, Jx); Jy, Jz: pair 1.  Words are 4 bytes,
        // like phi's elements, so phi's offsets address them.
        const gptr<const char> src0 = sbase(base);
        const gptr<const char> src1 = sbase(base + 2 * plane_bm);
#pragma unroll
        for (int j = 0; j < NPH; ++j) {
          const uint32_t w0 = *(gptr<const uint32_t>)(src0 + lane_off(phcol[j]));
          const uint32_t w1 = *(gptr<const uint32_t>)(src1 + lane_off(phcol[j]));
          v[0][j] = dec<R>(half_of<TM>(w0, 1), b.enc_off[1], b.enc_inv[1]);
          v[1][j] = dec<R>(half_of<TM>(w1, 0), b.enc_off[2], b.enc_inv[2]);
          v[2][j] = dec<R>(half_of<TM>(w1, 1), b.enc_off[3], b.enc_inv[3]);
        }
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const gptr<const char> src = sbase(base + (1 + a) * plane_bm);
#pragma unroll
          for (int j = 0; j < NPH; ++j) {
            const uint32_t off = phcol[j] / static_cast<uint32_t>(sizeof(TP)) * static_cast<uint32_t>(sizeof(TM));
            v[a][j] = dec<R>(*(gptr<const TM>)(src + lane_off(off)), b.enc_off[1 + a], b.enc_inv[1 + a]);
          }
        }
      }
    };
    // plane q lies beyond a z wall: every element of it is a ghost across that wall
    auto store_J = [&](R (*v)[NPH], int q) {
      const bool zflip = wz && (q < 0 || q >= nz);
#pragma unroll
      for (int j = 0; j < NPH; ++j) {
        const int e = tid + j * NT;
        if (j < NPH - 1 || e < NP) {
          const bool neg = (((jflip >> j) & 1u) != 0u) != zflip;
#pragma unroll
          for (int a = 0; a < 3; ++a) sh.jp[a * NP + e] = neg ? -v[a][j] : v[a][j];
        }
      }
    };
    // F[a] = (s_x s_y J_a, s_y d_x J_a, s_x d_y J_a, J_a at the centre)
    auto filter_J = [&](R (*F)[4]) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        R dx[3], sx[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const R* row = &sh.jp[a * NP + (ty + r) * PX + tx];
          const R l = row[0], c = row[1], h = row[2];
          dx[r] = h - l;
          sx[r] = l + R(4) * c + h;
          if (r == 1) F[a][3] = c;
        }
        F[a][0] = sx[0] + R(4) * sx[1] + sx[2];
        F[a][1] = dx[0] + R(4) * dx[1] + dx[2];
        F[a][2] = sx[2] - sx[0];
      }
    };

    R Fm[4], F0[4], Fp[4];
    R JFm[GC ? 3 : 1][4], JF0[GC ? 3 : 1][4], JFp[GC ? 3 : 1][4];
    R jnxt[GC ? 3 : 1][NPH];

    // moments of the own column, prefetched one plane ahead
    R nxt[NL];
    auto load_moments = [&](int q, R* m) {
      const gptr<const char> base = (gptr<const char>)s_mom + static_cast<int64_t>(map_plane(q, nz, wz)) * NM * plane_bm;
      if constexpr (PAIR) {
#pragma unroll
        for (int w = 0; w < (NL + 1) / 2; ++w) {
          const uint32_t v = *(gptr<const uint32_t>)(sbase(base + w * 2 * plane_bm) + lane_off(voff_w));
          m[2 * w] = dec<R>(half_of<TM>(v, 0), b.enc_off[2 * w], b.enc_inv[2 * w]);
          if (2 * w + 1 < NL) m[2 * w + 1] = dec<R>(half_of<TM>(v, 1), b.enc_off[2 * w + 1], b.enc_inv[2 * w + 1]);
        }
      } else {
#pragma unroll
        for (int k = 0; k < NL; ++k)
          m[k] = dec<R>(*(gptr<const TM>)(sbase(base + k * plane_bm) + lane_off(voff_m)), b.enc_off[k], b.enc_inv[k]);
      }
    };

    // The two planes staged before the march and the first prefetch are all
    // requested before any of them is used: an item then waits for memory
    // once up front instead of three times in a row (the in-order counter
    // lets each use wait only for the loads issued before it).
    R ph0[NPH], ph1[NPH];
    R jq0[GC ? 3 : 1][NPH], jq1[GC ? 3 : 1][NPH];
    load_phi(p_first - 1, ph0);
    if constexpr (GC) load_J(p_first - 1, jq0);
    load_phi(p_first, ph1);
    if constexpr (GC) load_J(p_first, jq1);
    load_moments(p_first, nxt);
    R phinxt[NPH];
    load_phi(p_first + 1, phinxt);
    if constexpr (GC) load_J(p_first + 1, jnxt);

    store_phi(ph0);
    if constexpr (GC) store_J(jq0, p_first - 1);
    __syncthreads();
    filter_phi(Fm);
    if constexpr (GC) filter_J(JFm);
    __syncthreads();
    store_phi(ph1);
    if constexpr (GC) store_J(jq1, p_first);
    __syncthreads();
    filter_phi(F0);
    if constexpr (GC) filter_J(JF0);
    __syncthreads();

    // Prefetched registers are consumed here, before this plane's global
    // stores are issued: loads and stores retire through one in-order vector
    // memory counter, so a wait placed after the stores (where the compiler
    // would put it, at the copy into next plane's registers) also waits for
    // every store.
    auto settle_prefetch = [&]() {
#pragma unroll
      for (int k = 0; k < NL; ++k) asm volatile("" ::"v"(nxt[k]));
#pragma unroll
      for (int j = 0; j < NPH; ++j) asm volatile("" ::"v"(phinxt[j]));
      if constexpr (GC) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int j = 0; j < NPH; ++j) asm volatile("" ::"v"(jnxt[a][j]));
      }
    };

    // The loop header joins this path with the back edge, where the prefetched
    // registers are already settled; settling them here too keeps the
    // compiler from placing a wait for them at the top of every iteration,
    // which (counting in order) would also wait for the previous plane's
    // stores.
    settle_prefetch();

    Acc<R> accM, acc0, accP;
    accM.zero();
    acc0.zero();
    R dM = R(0), d0 = R(0), dP = R(0);
    R phiH = R(0), lapH = R(0), advH = R(0);  // own-node phi, lap(phi), u.grad(phi) of plane p-1

    auto finalize = [&](int Z, const Acc<R>& a, R d, R phic, R lapc, R advc) {
      const gptr<char> base = (gptr<char>)d_mom + static_cast<int64_t>(Z) * NM * plane_bm;
      const R P = a.p;
      const R q_xx = a.xx - P * R(1.0 / 3.0) - a.jx * a.jx;
      const R q_yy = a.yy - P * R(1.0 / 3.0) - a.jy * a.jy;
      const R q_zz = a.zz - P * R(1.0 / 3.0) - a.jz * a.jz;
      const R q_xy = a.xy - a.jx * a.jy;
      const R q_xz = a.xz - a.jx * a.jz;
      const R q_yz = a.yz - a.jy * a.jz;
      const R phin = phic + mob * lapc - advc - d * R(1.0 / 72.0);
      const R mv[10] = {P, a.jx, a.jy, a.jz, q_xx, q_yy, q_zz, q_xy, q_xz, q_yz};
      // ZO: every 16-bit offset is +0 (the default encoding), so the encode
      // skips the subtraction of zeros (bitwise the same words)
      auto emit = [&](auto nt, auto zo) {
        constexpr bool N = decltype(nt)::value;
        constexpr bool ZO = decltype(zo)::value;
        store_out<N>((gptr<TP>)(sbase((gptr<char>)d_phi_g + static_cast<int64_t>(Z) * plane_bp) + lane_off(voff_p)),
                     Enc<TP>::go(phin, 0.f, 1.f));
        if constexpr (PAIR) {
#pragma unroll
          for (int w = 0; w < NM / 2; ++w)
            store_out<N>((gptr<uint32_t>)(sbase(base + w * 2 * plane_bm) + lane_off(voff_w)),
                         encode_pair<TM, ZO>(mv[2 * w], mv[2 * w + 1], b.enc_off[2 * w], b.enc_scale[2 * w],
                                             b.enc_off[2 * w + 1], b.enc_scale[2 * w + 1]));
        } else {
#pragma unroll
          for (int k = 0; k < NM; ++k)
            store_out<N>((gptr<TM>)(sbase(base + k * plane_bm) + lane_off(voff_m)),
                         Enc<TM>::go(mv[k], b.enc_off[k], b.enc_scale[k]));
        }
      };
      auto emit_enc = [&](auto nt) {
        if constexpr (PAIR) {
          if (b.zero_offsets) emit(nt, std::true_type{});
          else emit(nt, std::false_type{});
        } else {
          emit(nt, std::false_type{});
        }
      };
      if constexpr (NTS) {
        if (b.whole_rows) emit_enc(std::true_type{});
        else emit_enc(std::false_type{});
      } else {
        emit_enc(std::false_type{});
      }
    };

    for (int p = p_first; p <= p_last; ++p) {
      R cur[NL];
#pragma unroll
      for (int k = 0; k < NL; ++k) cur[k] = nxt[k];
      if (p < p_last) load_moments(p + 1, nxt);

      // (A) phi plane p+1 (prefetched) -> LDS -> filtered registers; prefetch p+2
      store_phi(phinxt);
      if (p < p_last) load_phi(p + 2, phinxt);
      if constexpr (GC) {
        store_J(jnxt, p + 1);
        if (p < p_last) load_J(p + 2, jnxt);
      }
      __syncthreads();
      filter_phi(Fp);
      if constexpr (GC) filter_J(JFp);

      // (B) node quantities at (column, p)
      const R phi = F0[3];
      R gx = (Fm[1] + R(4) * F0[1] + Fp[1]) * R(1.0 / 72.0);
      R gy = (Fm[2] + R(4) * F0[2] + Fp[2]) * R(1.0 / 72.0);
      const R gz = (Fp[0] - Fm[0]) * R(1.0 / 72.0);
      const R lap = (Fm[0] + R(4) * F0[0] + Fp[0]) * R(1.0 / 36.0) - R(6) * phi;
      uint32_t lf = lflags0;
      asm volatile("" : "+v"(lf));  // keep lane predicates in a VGPR, not hoisted masks
      const bool gcx = (lf & 1u) != 0, gcy = (lf & 2u) != 0;
      // gradient seen from the mirrored node (ghost columns of wall axes)
      const R gmx = gcx ? -gx : gx;
      const R gmy = gcy ? -gy : gy;

      const R P = cur[0];
      R Jx, Jy, Jz;
      if constexpr (GC) {
        // own J from the centre of the staged patch, which a ghost lane holds
        // with the sign (-1)^(walls crossed)
        const R so = (gcx != gcy) ? R(-1) : R(1);
        Jx = so * JF0[0][3];
        Jy = so * JF0[1][3];
        Jz = so * JF0[2][3];
      } else {
        Jx = cur[1 % NL];
        Jy = cur[2 % NL];
        Jz = cur[3 % NL];
      }

      // density, viscosity and relaxation interpolation (Sec. II.C),
      // evaluated at phi clamped to the model's range [0, 1]
      const R phid = fmin(fmax(phi, R(0)), R(1));
      const R drho = static_cast<R>(b.drho);
      const R rho = static_cast<R>(b.rho_g) + phid * drho;
      const R nu = static_cast<R>(b.nu_g) + phid * static_cast<R>(b.dnu);
      const R tau = R(3) * nu + R(0.5);  // 1 / omega
      const R r_rt = rcp_newton(rho * tau);  // one reciprocal for 1/rho and omega
      const R irho = tau * r_rt;
      const R om_d = rho * r_rt;
      const R bf = R(1) - static_cast<R>(b.rho_ref) * irho;  // body acceleration factor
      const R om1 = R(1) - om_d;
      const R cvis = R(-3) * nu * om_d * drho * irho;

      // The tensor the viscous correction contracts: the stored Q, or for the
      // gradient closure a2 itself, -(cs^2/omega)(d_a J_b + d_b J_a) with the
      // isotropic gradient of J (filtered planes p-1, p, p+1).  A ghost lane
      // (halo column beyond an x/y wall) sees J reflected with sign
      // s = (-1)^(walls crossed); the mirror node's gradient is its own times
      // s, and times -1 again along each crossed axis.
      R Txx, Tyy, Tzz, Txy, Txz, Tyz;
      if constexpr (GC) {
        R gJ[3][3];  // gJ[a][c] = d_c J_a
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          gJ[a][0] = (JFm[a][1] + R(4) * JF0[a][1] + JFp[a][1]) * R(1.0 / 72.0);
          gJ[a][1] = (JFm[a][2] + R(4) * JF0[a][2] + JFp[a][2]) * R(1.0 / 72.0);
          gJ[a][2] = (JFp[a][0] - JFm[a][0]) * R(1.0 / 72.0);
        }
        const R sg = (gcx != gcy) ? R(-1) : R(1);
        const R sdx = gcx ? -sg : sg, sdy = gcy ? -sg : sg;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          gJ[a][0] *= sdx;
          gJ[a][1] *= sdy;
          gJ[a][2] *= sg;
        }
        const R ca = -tau * R(1.0 / 3.0);  // -cs^2 / omega
        Txx = ca * (gJ[0][0] + gJ[0][0]);
        Tyy = ca * (gJ[1][1] + gJ[1][1]);
        Tzz = ca * (gJ[2][2] + gJ[2][2]);
        Txy = ca * (gJ[0][1] + gJ[1][0]);
        Txz = ca * (gJ[0][2] + gJ[2][0]);
        Tyz = ca * (gJ[1][2] + gJ[2][1]);
      } else {
        Txx = cur[4 % NL];
        Tyy = cur[5 % NL];
        Tzz = cur[6 % NL];
        Txy = cur[7 % NL];
        Txz = cur[8 % NL];
        Tyz = cur[9 % NL];
      }

      // chemical potential and the force per unit mass a = F / rho
      const R mu = beta4 * phi * (phi - R(1)) * (phi - R(0.5)) - kappa_mu * lap;
      const R csp = (mu - P * drho3) * irho;  // (F^s + F^p) / rho on grad(phi)
      const R qgx = Txx * gmx + Txy * gmy + Txz * gz;
      const R qgy = Txy * gmx + Tyy * gmy + Tyz * gz;
      const R qgz = Txz * gmx + Tyz * gmy + Tzz * gz;
      const R ax = csp * gmx + cvis * qgx + grx * bf;
      const R ay = csp * gmy + cvis * qgy + gry * bf;
      const R az = csp * gz + cvis * qgz + grz * bf;
      const R ux = Jx + R(0.5) * ax;
      const R uy = Jy + R(0.5) * ay;
      const R uz = Jz + R(0.5) * az;

      // a2 = Q + J J - u u + (u a + a u)/2 = Q + a a / 4 (moment closure), or
      // the gradient closure's a2 as it is
      const R Axx = GC ? Txx : Txx + R(0.25) * ax * ax;
      const R Ayy = GC ? Tyy : Tyy + R(0.25) * ay * ay;
      const R Azz = GC ? Tzz : Tzz + R(0.25) * az * az;
      const R Axy = GC ? Txy : Txy + R(0.25) * ax * ay;
      const R Axz = GC ? Txz : Txz + R(0.25) * ax * az;
      const R Ayz = GC ? Tyz : Tyz + R(0.25) * ay * az;

      // monomial coefficients of g(c) = f_post(c) / w(c), pre-scaled by 1/216,
      // written with B = (1 - omega) a2 and S_aa = u_a^2 + B_aa.  The relaxed
      // part of the first-order coefficients combines as
      // 13.5 u_x A_xx - 4.5 u_x tr(A) - 9 (A u)_x = -4.5 u_x (A_yy + A_zz)
      // - 9 (A_xy u_y + A_xz u_z), and likewise for y and z.
      const R Bxx = om1 * Axx, Byy = om1 * Ayy, Bzz = om1 * Azz;
      const R Bxy = om1 * Axy, Bxz = om1 * Axz, Byz = om1 * Ayz;
      const R Sxx = ux * ux + Bxx, Syy = uy * uy + Byy, Szz = uz * uz + Bzz;
      const R Exx = Sxx + ux * ax, Eyy = Syy + uy * ay, Ezz = Szz + uz * az;
      constexpr R s = R(1.0 / 216.0);
      const R G0 = s * P - (R(1.5) * s) * (Exx + Eyy + Ezz);
      const R Gx = s * (R(3) * ux + R(1.5) * ax) - (R(4.5) * s) * (ux * (Syy + Szz) + R(2) * (Bxy * uy + Bxz * uz));
      const R Gy = s * (R(3) * uy + R(1.5) * ay) - (R(4.5) * s) * (uy * (Sxx + Szz) + R(2) * (Bxy * ux + Byz * uz));
      const R Gz = s * (R(3) * uz + R(1.5) * az) - (R(4.5) * s) * (uz * (Sxx + Syy) + R(2) * (Bxz * ux + Byz * uy));
      const R Gxx = (R(4.5) * s) * Exx;
      const R Gyy = (R(4.5) * s) * Eyy;
      const R Gzz = (R(4.5) * s) * Ezz;
      const R hx = R(0.5) * ax, hy = R(0.5) * ay, hz = R(0.5) * az;
      const R Gxy = (R(9) * s) * (ux * (uy + hy) + (uy * hx + Bxy));
      const R Gxz = (R(9) * s) * (ux * (uz + hz) + (uz * hx + Bxz));
      const R Gyz = (R(9) * s) * (uy * (uz + hz) + (uz * hy + Byz));
      constexpr R s3 = R(13.5 / 216.0);
      const R Gxxy = s3 * (uy * Sxx + R(2) * (ux * Bxy));
      const R Gxxz = s3 * (uz * Sxx + R(2) * (ux * Bxz));
      const R Gyyx = s3 * (ux * Syy + R(2) * (uy * Bxy));
      const R Gyyz = s3 * (uz * Syy + R(2) * (uy * Byz));
      const R Gzzx = s3 * (ux * Szz + R(2) * (uz * Bxz));
      const R Gzzy = s3 * (uy * Szz + R(2) * (uz * Byz));
      const R Gxyz = R(27.0 / 216.0) * (ux * (uy * uz + Byz) + (uy * Bxz + uz * Bxy));

      // evaluate g(c) / 216 at the 27 velocities: x, then y, then z.  The
      // lattice weights w(c) = (1, 4, 1) x (1, 4, 1) x (1, 4, 1) / 216 are
      // applied where the pulled populations are summed (accum_group), as
      // multiply-adds that replace plain adds there.
      auto xb = [](R c0, R c1, R c2, R* o) { o[0] = c0 - c1 + c2; o[1] = c0; o[2] = c0 + c1 + c2; };
      auto xb2 = [](R c0, R c1, R* o) { o[0] = c0 - c1; o[1] = c0; o[2] = c0 + c1; };
      auto xb1 = [](R c0, R* o) { o[0] = c0; o[1] = c0; o[2] = c0; };
      R B00[3], B01[3], B02[3], B10[3], B11[3], B12[3], B20[3], B21[3];
      xb(G0, Gx, Gxx, B00);
      xb(Gy, Gxy, Gxxy, B01);
      xb2(Gyy, Gyyx, B02);
      xb(Gz, Gxz, Gxxz, B10);
      xb2(Gyz, Gxyz, B11);
      xb1(Gyyz, B12);
      xb2(Gzz, Gzzx, B20);
      xb1(Gzzy, B21);
      R fo[3];  // own column (cx, cy) = (0, 0), cz = -1, 0, 1
#pragma unroll
      for (int cyi = 0; cyi < 3; ++cyi) {
#pragma unroll
        for (int cxi = 0; cxi < 3; ++cxi) {
          const int cy = cyi - 1, cx = cxi - 1;
          R p0, p1, p2;
          if (cy == 0) {
            p0 = B00[cxi];
            p1 = B10[cxi];
            p2 = B20[cxi];
          } else {
            p0 = B00[cxi] + B02[cxi] + (cy > 0 ? B01[cxi] : -B01[cxi]);
            p1 = B10[cxi] + B12[cxi] + (cy > 0 ? B11[cxi] : -B11[cxi]);
            p2 = B20[cxi] + (cy > 0 ? B21[cxi] : -B21[cxi]);
          }
          const R fm = p0 + p2 - p1;  // cz = -1
          const R f0 = p0;            // cz = 0
          const R fp = p0 + p2 + p1;  // cz = +1
          if (cx == 0 && cy == 0) {
            fo[0] = fm;
            fo[1] = f0;
            fo[2] = fp;
          } else {
            sh.f[fslot(cx, cy, -1) * NT + sp] = fm;
            sh.f[fslot(cx, cy, 0) * NT + sp] = f0;
            sh.f[fslot(cx, cy, 1) * NT + sp] = fp;
          }
        }
      }

      // phase-field flux G at this node (ghost rules on mirrored columns)
      {
        const R ig = inv_norm_eps(gx * gx + gy * gy + gz * gz);  // 1 / (|grad phi| + 1e-12)
        const R sharp = kappa_ac * phi * (R(1) - phi) * ig;
        const R us = (gcx != gcy) ? R(-1) : R(1);
        const R pu = literal ? R(0) : phi * us;
        const R Gfx = pu * ux + sharp * gx;
        const R Gfy = pu * uy + sharp * gy;
        const R Gfz = pu * uz + sharp * gz;
        sh.g[0 * NT + sp] = Gfx;
        sh.g[1 * NT + sp] = Gfy;
        sh.g[2 * NT + sp] = Gfz;
        if (wz && (p == 0 || p == nz - 1)) {
          // ghost plane beyond the z wall: velocity reversed, n_z reversed
          sh.gg[0 * NT + sp] = -pu * ux + sharp * gx;
          sh.gg[1 * NT + sp] = -pu * uy + sharp * gy;
          sh.gg[2 * NT + sp] = -pu * uz - sharp * gz;
        }
      }
      const R adv_own = literal ? (ux * gmx + uy * gmy + uz * gz) : R(0);
      settle_prefetch();
      // ghost columns contribute no regular pulls: the populations that would
      // stream out of them are replaced by bounce-back at the wall node
      if (wall_tile && (gcx || gcy)) {
#pragma unroll
        for (int k = 0; k < 24; ++k) sh.f[k * NT + sp] = R(0);
      }
      __syncthreads();

      // (C) pull, accumulate, finalise output plane p-1
      if (out_col) {
        const bool zb_lo = wz && p == 0;
        const bool zb_hi = wz && p == nz - 1;
        // regular pulls from the 3 x 3 neighbour columns
#pragma unroll
        for (int czi = 0; czi < 3; ++czi) {
          R v[9];
#pragma unroll
          for (int k = 0; k < 9; ++k) {
            const int cx = k % 3 - 1, cy = k / 3 - 1;
            if (k == 4) v[k] = fo[czi];
            else v[k] = sh.f[fslot(cx, cy, czi - 1) * NT + sp - cy * BX - cx];
          }
          if (czi == 0) accum_group<R, -1>(v, accM);
          else if (czi == 1) accum_group<R, 0>(v, acc0);
          else accum_group<R, 1, true>(v, accP);
        }
        // half-way bounce-back into this node (plane p): direction c pulls from
        // behind a wall when the node is on that wall's side, and then takes
        // the node's own post-collision population of direction -c
        if (wall_tile || zb_lo || zb_hi) {
          uint32_t lw = lflags0;
          asm volatile("" : "+v"(lw));
#pragma unroll
          for (int czi = 0; czi < 3; ++czi) {
            const int cz = czi - 1;
            const bool zb = (zb_lo && cz == 1) || (zb_hi && cz == -1);
            R v[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
              const int cx = k % 3 - 1, cy = k / 3 - 1;
              const uint32_t m = (cx > 0 ? 4u : 0u) | (cx < 0 ? 8u : 0u) | (cy > 0 ? 16u : 0u) | (cy < 0 ? 32u : 0u);
              const bool behind = zb || (lw & m) != 0u;
              R own;
              if (k == 4) own = fo[2 - czi];
              else own = sh.f[fslot(-cx, -cy, -cz) * NT + sp];
              v[k] = behind ? own : R(0);
            }
            if (czi == 0) accum_group<R, -1>(v, acc0);
            else if (czi == 1) accum_group<R, 0>(v, acc0);
            else accum_group<R, 1>(v, acc0);
          }
        }
        // divergence of the phase-field flux (forward neighbours x + c)
        {
          auto G = [&](int comp, int cx, int cy) { return sh.g[comp * NT + sp + cy * BX + cx]; };
          R hx, hy, hz;
          div_sums(G, hx, hy, hz);
          const R hxy = hx + hy;
          dM += hxy + hz;
          d0 += R(4) * hxy;
          dP = hxy - hz;
          if (zb_lo || zb_hi) {
            auto GG = [&](int comp, int cx, int cy) { return sh.gg[comp * NT + sp + cy * BX + cx]; };
            R gx2, gy2, gz2;
            div_sums(GG, gx2, gy2, gz2);
            // plane -1 feeds output 0 with (Hxy - Hz); plane nz feeds nz-1 with (Hxy + Hz)
            if (zb_lo) d0 += (gx2 + gy2) - gz2;
            if (zb_hi) d0 += (gx2 + gy2) + gz2;
          }
        }
        if (p - 1 >= z0 && p - 1 < z1) finalize(p - 1, accM, dM, phiH, lapH, advH);
        accM = acc0;
        acc0 = accP;
        dM = d0;
        d0 = dP;
        phiH = phi;
        lapH = lap;
        advH = adv_own;
      }
      // rotate the filtered phi planes
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        Fm[k] = F0[k];
        F0[k] = Fp[k];
      }
      if constexpr (GC) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            JFm[a][k] = JF0[a][k];
            JF0[a][k] = JFp[a][k];
          }
      }
    }
    // top wall: the last node plane is the last output plane
    if (out_col && wz && z1 == nz) finalize(nz - 1, accM, dM, phiH, lapH, advH);
    __syncthreads();
  }
}

template <int BX, int BY, class PR, bool GC>
hipError_t launch_fused_t(const BoxDesc* d_boxes, const Item* d_items, int n_items, int grid, int parity,
                          hipStream_t stream) {
  hipLaunchKernelGGL((fused_step<BX, BY, PR, GC>), dim3(grid), dim3(BX * BY), 0, stream, d_boxes, d_items,
                     n_items, parity);
  return hipGetLastError();
}

template <int BX, int BY, class PR, bool GC>
int fused_blocks_per_cu_t() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fused_step<BX, BY, PR, GC>, BX * BY, 0) != hipSuccess) return 0;
  return n;
}

template <int BX, int BY, bool GC>
int fused_blocks_per_cu_t(int precision) {
  switch (precision) {
    case kF64: return fused_blocks_per_cu_t<BX, BY, PF64, GC>();
    case kF32: return fused_blocks_per_cu_t<BX, BY, PF32, GC>();
    case kF16: return fused_blocks_per_cu_t<BX, BY, PF16, GC>();
    case kBF16: return fused_blocks_per_cu_t<BX, BY, PBF16, GC>();
    default: return 0;
  }
}

template <int BX, int BY, bool GC>
hipError_t launch_fused_t(int precision, const BoxDesc* d_boxes, const Item* d_items, int n_items,
                          int grid, int parity, hipStream_t stream) {
  return dispatch(precision, [&](auto pr) {
    using PR = decltype(pr);
    return launch_fused_t<BX, BY, PR, GC>(d_boxes, d_items, n_items, grid, parity, stream);
  });
}

}  // namespace


// Tile shapes: (32,8) (34,8) (34,15) for both closures and every precision;
// (18,14) for the moment closure; (66,8) for the moment closure outside FP64
// (FP64 needs > 168 VGPRs there: it would spill).
bool fused_config_supported(int precision, bool gc, int bx, int by) {
  if ((bx == 32 && by == 8) || (bx == 34 && by == 8) || (bx == 34 && by == 15)) return true;
  if (gc) return false;
  if (bx == 18 && by == 14) return true;
  return bx == 66 && by == 8 && precision != kF64;
}

size_t phi_bytes(int precision, int64_t n) { return static_cast<size_t>(n) * (precision == kF64 ? 8 : 4); }
int row_pitch(int precision, int nx) {
  const int e = precision == kF64 ? 8 : (precision == kF32 ? 4 : 2);  // smaller of the phi and moment sizes
  const int q = 64 / e;
  return (nx + q - 1) / q * q;
}
size_t mom_bytes(int precision, int64_t n, int nmom) {
  const size_t e = precision == kF64 ? 8 : (precision == kF32 ? 4 : 2);
  return static_cast<size_t>(n) * static_cast<size_t>(nmom) * e;
}

int fused_blocks_per_cu(int precision, bool gc, int bx, int by) {
  if (!fused_config_supported(precision, gc, bx, by)) return 0;
  if (gc) {
    if (bx == 32 && by == 8) return fused_blocks_per_cu_t<32, 8, true>(precision);
    if (bx == 34 && by == 8) return fused_blocks_per_cu_t<34, 8, true>(precision);
    return fused_blocks_per_cu_t<34, 15, true>(precision);
  }
  if (bx == 32 && by == 8) return fused_blocks_per_cu_t<32, 8, false>(precision);
  if (bx == 34 && by == 8) return fused_blocks_per_cu_t<34, 8, false>(precision);
  if (bx == 34 && by == 15) return fused_blocks_per_cu_t<34, 15, false>(precision);
  if (bx == 18 && by == 14) return fused_blocks_per_cu_t<18, 14, false>(precision);
  if (precision == kF32) return fused_blocks_per_cu_t<66, 8, PF32, false>();
  if (precision == kF16) return fused_blocks_per_cu_t<66, 8, PF16, false>();
  return fused_blocks_per_cu_t<66, 8, PBF16, false>();
}

hipError_t launch_fused(int precision, bool gc, int bx, int by, const BoxDesc* d_boxes, const Item* d_items,
                        int n_items, int grid, int parity, hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  if (!fused_config_supported(precision, gc, bx, by)) return hipErrorInvalidValue;
  if (grid <= 0 || grid > n_items) grid = n_items;
  if (gc) {
    if (bx == 32 && by == 8) return launch_fused_t<32, 8, true>(precision, d_boxes, d_items, n_items, grid, parity, stream);
    if (bx == 34 && by == 8) return launch_fused_t<34, 8, true>(precision, d_boxes, d_items, n_items, grid, parity, stream);
    return launch_fused_t<34, 15, true>(precision, d_boxes, d_items, n_items, grid, parity, stream);
  }
  if (bx == 32 && by == 8) return launch_fused_t<32, 8, false>(precision, d_boxes, d_items, n_items, grid, parity, stream);
  if (bx == 34 && by == 8) return launch_fused_t<34, 8, false>(precision, d_boxes, d_items, n_items, grid, parity, stream);
  if (bx == 34 && by == 15) return launch_fused_t<34, 15, false>(precision, d_boxes, d_items, n_items, grid, parity, stream);
  if (bx == 18 && by == 14) return launch_fused_t<18, 14, false>(precision, d_boxes, d_items, n_items, grid, parity, stream);
  if (bx == 66 && by == 8) {
    if (precision == kF32) return launch_fused_t<66, 8, PF32, false>(d_boxes, d_items, n_items, grid, parity, stream);
    if (precision == kF16) return launch_fused_t<66, 8, PF16, false>(d_boxes, d_items, n_items, grid, parity, stream);
    return launch_fused_t<66, 8, PBF16, false>(d_boxes, d_items, n_items, grid, parity, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm
