// Internal declarations of libnmg: device-side descriptors and the kernel launchers shared by
// the translation units.  Not part of the public ABI (include/nmg.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nmg.h"

namespace nmg {

constexpr int kTile = 256;        // threads (= cells) per 1D tile
constexpr int kCoarsenCells = 4;  // level-l0 cells per thread in the coarsening kernel
constexpr int kMaxLevels = 16;
constexpr int kMaxCoarse = 256;   // cells on the coarsest 1D level (one thread per cell)
constexpr int kBottomThreads = 1024;          // threads of the bottom-of-cycle kernel
constexpr int kBottomCells = 2 * kBottomThreads;  // largest level it handles
constexpr double kZeta = 1e-6;    // WENO epsilon of eq. (8)

// One 1D instance as the kernels see it.
struct Inst1D {
    int N, levels, nb, active_idx;   // active_idx: index of this instance's NewtonState
    double dx, g;
    int bc_kind[2];
    double bc_q[2], bc_h[2];
    const double *sig_face, *sig_gp, *sigx_gp, *bx_gp;
    double *U;         // state [2][N] (caller memory)
    double *R;         // residual [2][N]
    double *rn;        // ||R_j||_1 [N]
    double alpha, tau, eps, omega, tol;
    int nu1, nu2, nu3, n_max;
    int lev0;          // index of level 0 in the level table
    int levc;          // index of the coarsest level
    int res_tile0, res_tiles;  // residual tiles of this instance (contiguous)
    int max_hist;
    int lbot;          // first level handled by the bottom-of-cycle kernel
    double *hist;      // device history of res, [max_hist] (may be null)
};

// One multigrid level of one instance.  Offsets are in elements of the MG value type.
struct Level1D {
    int inst, l, n, nb;
    int coarsest, halo, V, child;    // child: level index of l+1 (-1 at the coarsest)
    long long J, Dinv, rhs, dU;
};

struct Tile {
    int lev;   // instance index (residual/Jacobian tiles) or level index (multigrid tiles)
    int a;     // first cell of the tile's valid range
};

struct NewtonState {
    double res;
    int n, active, status, pad;
};

// Kernel arguments common to the multigrid kernels.
struct MGArgs {
    const Inst1D *insts;
    const Level1D *levs;
    NewtonState *state;   // may be null: every instance active
    void *mg;             // base of the multigrid value arrays (double or float)
};

__host__ __device__ inline int halo_cells(int nb, int nu)
{
    // one symmetric step = 2C half-sweeps; each moves information nb/2 cells
    int C = nb == 5 ? 3 : 2;
    return nu * 2 * C * (nb / 2);
}

// ---- launchers (return hipError_t of the launch) ----------------------------------------

// residual over tiles (batched: tiles index instances) or one instance (tiles == null)
hipError_t launch_residual1d(const Inst1D *insts_dev, const Tile *tiles, int ntiles,
                             const Inst1D *single, NewtonState *state, double *partial,
                             hipStream_t s);
hipError_t launch_res_finalize(const Inst1D *insts_dev, int ninst, NewtonState *state,
                               const double *partial, int init, hipStream_t s);
hipError_t launch_sum_res(const double *rn, int N, double *res, hipStream_t s);
// Jacobian: writes FP64 (prec 0) or FP32 (prec 1) blocks with row stride N at J_out (single) or
// at each instance's level-0 J (batched, via the level table)
hipError_t launch_jacobian1d(const Inst1D *insts_dev, const Tile *tiles, int ntiles,
                             const Inst1D *single, double *J_single, const MGArgs &mg, int prec,
                             int nb_mask, hipStream_t s);
hipError_t launch_coarsen1d(const MGArgs &mg, const Tile *tiles, int ntiles, int prec, hipStream_t s);
hipError_t launch_bottom(const MGArgs &mg, const int *inst_list, int n, int zero_init0, int final_update,
                         int prec, hipStream_t s);
hipError_t launch_smooth1d(const MGArgs &mg, const Tile *tiles, int ntiles, int nb_max, int mode,
                           int zero_init, int final_update, int prec, hipStream_t s);
hipError_t launch_convert(const void *src, int src_prec, void *dst, int dst_prec, long long n,
                          hipStream_t s);

}  // namespace nmg
