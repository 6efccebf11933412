// Internal interface between the C-ABI runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "eulbfs_device.h"

namespace eulbfs {

// Shu-Osher SSP-RK3 stage (Eq. 58): W_out = ca W^n + cb W^(k) + cc dt R(W^(k)).
struct StageCoef {
    double ca, cb, cc;
    int last;  // third stage: also write the lagged dF_s/dt
};

// Intermediate planes of the split path (ghosted grid of (nx+6) x (ny+6)).
template <typename R>
struct SplitScratch {
    State<R> g;      // ghosted conserved state
    int gpitch;
    R* prim;         // NPRIM + 1 planes (T, C, F_s, u, v, p, mu_c, rho), ghosted
    size_t pstride;  // elements between prim planes
    R* Fx;           // 5 planes, (ny) rows of fpitch, x-face i at column i
    R* Fy;           // 5 planes, (ny + 1) rows of fpitch
    int fpitch;
    size_t fstride;  // elements between flux planes
};

enum { TILE_32x8 = 0, TILE_64x4 = 1, TILE_16x16 = 2, TILE_64x8 = 3, TILE_32x16 = 4, TILE_32x32 = 5, NTILES = 6 };

constexpr int NXCD = 8;  // accelerator complex dies of an MI355X, each with its own L2

// Tiles of the batched stage kernel: the two shapes that led on the serving
// mix (grids of 64^2 to 512^2 in FP32 mode: 67 and 66 solves/s against 60 for
// 32 x 8 and 48 for 32 x 32).  A batch picks one of them by timing its own
// ticks; stretched meshes always take the first.
constexpr int NBATCH_TILES = 2;
constexpr int BATCH_TX[NBATCH_TILES] = {32, 64}, BATCH_TY[NBATCH_TILES] = {16, 8};

// Tile of the fused stage kernel on a stretched mesh, one shape per field
// type: 32 x 16 in FP64, where a 1024-thread 32 x 32 tile would need 162 KB of
// LDS and spill the mesh weights; 32 x 32 in FP32 (6-7 % faster than 32 x 16
// at 512^2).  The batched kernel runs stretched requests with its own tile;
// every tile shape gives the same bits.
template <typename R>
struct NuTile {
    static constexpr int TX = 32, TY = sizeof(R) == 4 ? 32 : 16;
};

// One request of a batch: its constants, its three copies of W (W^n, W1, W2)
// and its dF_s/dt plane, and where its tiles start in the batch's tile list.
template <typename R>
struct BatchDesc {
    DevParams P;
    State<R> W[3];
    R* fsdot;
    int tiles_x;
    int tile0;
};

// Slots of the FP64 reduction: sums of rho, C, H and F_s over the cells,
// max |u|, the count of non-finite cells, F_s and clamped C summed up the
// middle column (tip and axis heights), max of -C and of C, clamped C summed
// along the first row (wetted length on the y- wall).
enum {
    RED_RHO = 0, RED_C, RED_H, RED_FS, RED_UMAX, RED_NONFINITE, RED_TIP,
    RED_NEG_CMIN, RED_CMAX, RED_WALL, RED_AXIS, NRED
};

template <typename R>
hipError_t launch_stage_fused(const DevParams& P, int tile, const StageCoef& K, const State<R>& in,
                              const State<R>& Wn, const State<R>& out, R* fsdot, hipStream_t st);
template <typename R>
hipError_t launch_stage_split(const DevParams& P, const SplitScratch<R>& X, const StageCoef& K, const State<R>& in,
                              const State<R>& Wn, const State<R>& out, R* fsdot, R* resid, size_t resid_stride,
                              hipStream_t st);
template <typename R>
hipError_t launch_init(const DevParams& P, const double* prim6, const State<R>& out, R* fsdot, hipStream_t st);

// Closed-form initial primitive fields (the public eulbfs_shape; profile 0
// uniform, 1 layer, 2 droplet).
struct InitShape {
    int profile, axis;
    double c0, h0, x0, y0, r0, t_out, t_in, t_amp;
    uint64_t seed;
    double fl0, u_in, v_in, xi;
};
hipError_t launch_init_shape(const DevParams& P, const InitShape& S, double* prim6, hipStream_t st);
template <typename R>
hipError_t launch_set_conserved(const DevParams& P, const double* w6, const State<R>& out, R* fsdot, int which,
                                hipStream_t st);
template <typename R>
hipError_t launch_export(const DevParams& P, const State<R>& S, const R* fsdot, int what, double* dst,
                         hipStream_t st);
template <typename R>
hipError_t launch_stage_batched(const BatchDesc<R>* descs, const int* tile_req, int ntiles, int lattice, int fast,
                                bool nu, int tile, const StageCoef& K, int stage, hipStream_t st);
template <typename R>
hipError_t launch_reduce(const DevParams& P, const State<R>& S, double* partial, int nblocks, double* out,
                         hipStream_t st);

}  // namespace eulbfs
