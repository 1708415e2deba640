// Internal interface between the host runtime (runtime.cpp) and the device
// code (fused_step.hip, aux_kernels.hip, noalloc.hip) of liblbm.so.  Not part
// of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lbm.h"
#include "state_layout.h"

namespace lbm {



// Fused step over n_items tiles; reads buffer `parity`, writes 1 - parity.
// grid workgroups loop over the items with stride grid.
// gc selects the gradient-closure kernel (every box of the launch must use it).
hipError_t launch_fused(int precision, bool gc, int block_x, int block_y, const BoxDesc* d_boxes,
                        const Item* d_items, int n_items, int grid, int parity,
                        hipStream_t stream);
bool fused_config_supported(int precision, bool gc, int block_x, int block_y);
// Workgroups of the fused kernel that fit on one compute unit at once (0 on error).
int fused_blocks_per_cu(int precision, bool gc, int block_x, int block_y);

// Bytes of the phi and moment arrays of one buffer of a box of n nodes with
// nmom moment fields.
size_t phi_bytes(int precision, int64_t n);
size_t mom_bytes(int precision, int64_t n, int nmom);
// Stored row length (elements) for rows of nx nodes: nx rounded up so that
// rows of phi and of every moment field start on 64-byte boundaries.
int row_pitch(int precision, int nx);

// Encode N doubles into field `field` (storage of `precision`).
hipError_t launch_encode(int precision, const BoxDesc& box, int parity, int field,
                         const double* d_src, int64_t n, hipStream_t stream);
// Decode field `field` into N doubles.
hipError_t launch_decode(int precision, const BoxDesc& box, int parity, int field,
                         double* d_dst, int64_t n, hipStream_t stream);
// Gather the 11 decoded fields at n nodes: d_out[k*n + j] for node d_idx[j].
hipError_t launch_gather(int precision, const BoxDesc& box, int parity, const int64_t* d_idx, int64_t n,
                         double* d_out, hipStream_t stream);
// Observable `which` (0 rho, 1 ux, 2 uy, 3 uz, 4 phi, 5 p) into N doubles.
hipError_t launch_observable(int precision, const BoxDesc& box, int parity, int which,
                             double* d_dst, hipStream_t stream);

// Host-side helpers shared by the context API (runtime.cpp) and the entry
// point that allocates nothing (noalloc.hip).
// Parameter checks of lbm_create for box idx; on failure the message is the
// context-free error text (lbm_last_error(NULL)).
lbm_status check_params(const lbm_params& p, int idx, int precision0, const char* who);
// Set / clear the context-free error text; set_error returns s.
lbm_status set_error(lbm_status s, const char* fmt, ...);
void clear_error();
// -1 if every scale is a positive power of two and every offset finite;
// else k (scale[k] bad) or 10 + k (offset[k] bad).
int check_encoding(const double* offset, const double* scale);
// Offsets 0 and scales 1024 (P), 4096 (J), 65536 (Q).
void default_encoding(double off[10], double scale[10]);
// Descriptor of one box from its parameters; d.phi and d.mom must already
// hold the state buffers (their alignment decides d.whole_rows).
void fill_box_desc(const lbm_params& p, int precision, const double off[10], const double scale[10], BoxDesc& d);

// Fourth-order phase-field update of boxes box0 .. box0 + nbox - 1 (every
// one with LBM_HIGH_ORDER_AC and its aux planes; gc: they use the gradient
// closure; literal: they advect with the printed u . grad(phi)): reads state
// `parity`, overwrites phi of buffer 1 - parity.  Runs after the fused step of
// the same parity.  flux_blocks: workgroups per box of the flux kernel
// (high_order_blocks_per_box of the largest box); phase_tiles: the largest
// high_order_phase_tiles over the boxes.
hipError_t launch_high_order_phase(int precision, bool gc, bool literal, const BoxDesc* d_boxes, int box0, int nbox,
                                   int parity, int flux_blocks, int phase_tiles, hipStream_t stream);
int high_order_blocks_per_box(int64_t max_nodes);
int high_order_phase_tiles(int nx, int ny, int nz);

// Finer phase-field grid (LBM_FINE_PHASE), boxes with fphi / aux
// (3 planes) allocated.
// launch_fine_init: fine phi of buffer `parity` interpolated from the coarse
// phi, then the coarse phi replaced by the restriction (d_box: this box's
// device descriptor).  launch_fine_set: fine phi from 8 N doubles (fine
// layout [2nz][2ny][2nx]), then the restriction.  launch_fine_get: fine phi
// decoded into 8 N doubles.
hipError_t launch_fine_init(int precision, const BoxDesc& box, const BoxDesc* d_box, int parity, hipStream_t stream);
hipError_t launch_fine_set(int precision, const BoxDesc& box, const BoxDesc* d_box, int parity, const double* d_src,
                           hipStream_t stream);
hipError_t launch_fine_get(int precision, const BoxDesc& box, int parity, double* d_dst, hipStream_t stream);
// launch_fine_gather: the decoded fine phi at n flat fine indices d_idx
// (device, each in [0, 8 N)) into d_out.
hipError_t launch_fine_gather(int precision, const BoxDesc& box, int parity, const int64_t* d_idx, int64_t n,
                              double* d_out, hipStream_t stream);
// The phase update of a step on the fine grids of boxes box0 .. box0 + nbox
// - 1: reads level `parity` (coarse state and fine phi), writes the fine phi
// of buffer 1 - parity and overwrites the coarse phi of buffer 1 - parity
// with its restriction.  Runs after the fused step of the same parity.
// u_blocks: high_order_blocks_per_box of the largest box; step_tiles: the
// largest fine_tiles over the boxes (one workgroup per tile);
// restrict_blocks: workgroups per box of the restriction.
hipError_t launch_fine_phase(int precision, bool gc, const BoxDesc* d_boxes, int box0, int nbox, int parity,
                             int u_blocks, int step_tiles, int restrict_blocks, hipStream_t stream);
int fine_tiles(int nx, int ny, int nz);

constexpr int kDiagValues = 28;
constexpr int kDiagBlocks = 1024;
// Workgroups per box of the diagnostics launch for boxes of at most
// max_nodes nodes (at least 16 nodes per thread, at most kDiagBlocks).
int diag_blocks_per_box(int64_t max_nodes);
// FP64 reductions of boxes box0 .. box0 + nbox - 1 of the device descriptor
// array in one launch: partials (nbox * blocks_per_box * kDiagValues
// doubles), then kDiagValues doubles per box into d_out (box after box).  The
// order of every sum is fixed by blocks_per_box alone, so a box gives bitwise
// the same values whether it is reduced alone or with the others.
// gc: the boxes use the gradient closure (every box of a launch alike).
hipError_t launch_diagnostics(int precision, bool gc, const BoxDesc* d_boxes, int box0, int nbox, int parity,
                              int blocks_per_box, double* d_partials, double* d_out, hipStream_t stream);

}  // namespace lbm
