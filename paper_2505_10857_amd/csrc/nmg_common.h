// Internal declarations of libnmg: device-side descriptors and the kernel launchers shared by
// the translation units.  Not part of the public ABI (include/nmg.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nmg.h"

namespace nmg {

constexpr int kTile = 256;        // threads (= cells) per 1D tile
constexpr int kSmoothTile = 256;  // default threads (= cells) per tile of the tiled multigrid smoother
constexpr int kSmoothTileMax = 512;  // the other width the plan options offer
constexpr size_t kMemCacheBytes = size_t(256) << 20;   // MI355X memory-side (Infinity) cache
constexpr int kCoarsenCells = 4;  // level-l0 cells per thread in the coarsening kernel
constexpr int kMaxLevels = 16;
constexpr int kMaxCoarse = 256;   // cells on the coarsest 1D level (one thread per cell)
constexpr int kBottomCellsMax = 2048;  // largest level the bottom-of-cycle kernel handles
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
    int n_start;       // Newton steps already taken (a resumed instance); 0 for a fresh one
    int sor_tile0, sor_tiles;  // Newton-SOR tiles of this instance (contiguous)
    double *hist;      // device history of res, [max_hist] (may be null)
    int recon;         // NMG_RECON_CONSERVED or NMG_RECON_SURFACE (then the width is taken as 1)
    const double *z_face, *z_avg;   // surface reconstruction: bottom at faces [N+1], cell averages [N+4]
};

// One multigrid level of one instance.  Offsets are in elements of the MG value type.
struct Level1D {
    int inst, l, n, nb;
    int coarsest, halo, V, child;    // child: level index of l+1 (-1 at the coarsest)
    int halo2, V2;                   // halo and valid width of a launch running nu2 + nu1 steps
    long long J, rhs, dU;
    // second dU buffer [2][n]: a tiled kernel reads its tile and halo from one buffer and writes
    // its cells to the other, so that no workgroup reads a halo cell that a neighbouring tile of
    // the same launch has already overwritten
    long long dUo;
    long long aux;                   // Newton-SOR, level 0: dU before the current step [2][n]
};

struct Tile {
    int lev;   // instance index (residual/Jacobian tiles) or level index (multigrid tiles)
    int a;     // first cell of the tile's valid range
};

struct NewtonState {
    double res;
    int n, active, status;
    int sor_done;   // Newton-SOR: the inner SOR iteration of the current step has stopped
};

// Kernel arguments common to the multigrid kernels.
struct MGArgs {
    const Inst1D *insts;
    const Level1D *levs;
    NewtonState *state;   // may be null: every instance active
    void *mg;             // base of the multigrid value arrays (double or float)
};

// Halo of a tiled multigrid smoothing launch running nu_a then nu_b symmetric steps (k_smooth):
// the steps' runs of one colour (consecutive half-sweeps of a colour merged, nu (2C - 2) + 1
// runs for nu steps) each move information nb/2 cells, and the restriction reads the neighbours
// of every cell written once more.  A tile cell whose distance to the tile edge is at least
// this many cells holds the exact value of the untiled sweep.  The width is rounded up to even:
// a tile then starts at an even cell, which pairs the two children of a coarse cell in adjacent
// lanes (t, t ^ 1) for the restriction.
__host__ __device__ inline int smooth_halo(int nb, int nu_a, int nu_b)
{
    const int C = nb == 5 ? 3 : 2;
    auto runs = [C](int nu) { return nu > 0 ? nu * (2 * C - 2) + 1 : 0; };
    const int h = (runs(nu_a) + runs(nu_b) + 1) * (nb / 2);
    return (h + 1) & ~1;
}

__host__ __device__ inline int halo_cells(int nb, int nu)
{
    // one symmetric step = 2C half-sweeps; each moves information nb/2 cells
    int C = nb == 5 ? 3 : 2;
    return nu * 2 * C * (nb / 2);
}

// One 2D instance (section 4).
struct Inst2D {
    int Nx, Ny;
    double dx, dy, g, x0, y0;
    int bc_kind[4];
    double bc_q[4], bc_h[4], bc_u[4], bc_v[4];
    double wall_x;
    const double *bx, *by;     // [Ny][Nx][2][2]: (y point beta, x point gamma)
    double *U, *R, *rn;        // U, R: [3][Ny][Nx]
    double alpha, eps;
    // surface reconstruction (recon = NMG_RECON_SURFACE): cell averages of b over cells
    // -2..Nx+1 x -2..Ny+1 ([Ny+4][Nx+4]), b at the two Gauss points of every x face
    // ([Ny][Nx+1][2]) and of every y face ([Ny+1][Nx][2])
    int recon;
    const double *zavg, *zfx, *zfy;
};

// Colour-blocked cell order of a 2D level: the cells of one colour are stored together, row by
// row, so that a colour pass of the smoother reads contiguous data.  C = 2 or 3: colour
// c = (i + j) mod C, cell (i, j) at c*ny*W + j*W + (i - i_c(j)) / C, i_c(j) the first column of
// colour c in row j and W = ceil(nx / C) slots per row and colour.  C = 9 (the full 21-cell
// stencil): colour c = (i mod 3) + 3 (j mod 3), cell (i, j) at c*ceil(ny/3)*W + (j/3)*W + i/3 with
// W = ceil(nx / 3).  C = 1 is the natural order j*nx + i.
struct Perm2D {
    int C, W, ny, pad;  // ny: rows per colour (ny of the level, ceil(ny / 3) when C = 9)
    long long M;       // slots per array: C * ny * W
};

__host__ __device__ inline long long perm2d(const Perm2D &P, int i, int j)
{
    if (P.C == 9) return (long long)(i % 3 + 3 * (j % 3)) * P.ny * P.W + (long long)(j / 3) * P.W + i / 3;
    const int c = (i + j) % P.C;
    const int ic = ((c - j) % P.C + P.C) % P.C;
    return (long long)c * P.ny * P.W + (long long)j * P.W + (i - ic) / P.C;
}

inline Perm2D make_perm2d(int nx, int ny, int C)
{
    Perm2D P;
    P.C = C;
    P.W = C == 9 ? (nx + 2) / 3 : (nx + C - 1) / C;
    P.ny = C == 9 ? (ny + 2) / 3 : ny;
    P.pad = 0;
    P.M = (long long)C * P.ny * P.W;
    return P;
}

// Block b of a 2D stencil of nb blocks (closed forms, no tables): nb = 9, the cross of eq. (21)
// (centre, x-2, x-1, x+1, x+2, y-2, y-1, y+1, y+2); nb = 21, the full stencil (the cross, then
// x-2, x-1, x+1, x+2 on row y-1 and on row y+1, then x-1 and x+1 on rows y-2 and y+2, the row
// first); nb = 5, the five points of the coarse levels (centre, x-1, x+1, y-1, y+1).
__host__ __device__ constexpr int stencil_dx(int nb, int b)
{
    if (nb == 5) return b == 1 ? -1 : (b == 2 ? 1 : 0);
    if (b < 9) return (b >= 1 && b <= 4) ? (b <= 2 ? b - 3 : b - 2) : 0;
    if (b < 17) return ((b - 9) & 3) < 2 ? ((b - 9) & 3) - 2 : ((b - 9) & 3) - 1;
    return b - 17 < 2 ? -1 : 1;
}
__host__ __device__ constexpr int stencil_dy(int nb, int b)
{
    if (nb == 5) return b == 3 ? -1 : (b == 4 ? 1 : 0);
    if (b < 9) return b >= 5 ? (b <= 6 ? b - 7 : b - 6) : 0;
    if (b < 17) return b - 9 < 4 ? -1 : 1;
    return ((b - 17) & 1) ? 2 : -2;
}

// One 2D multigrid level: blocks J [nb*9][M], Dinv [9][M], rhs [3][M], dU [3][M] in the level's
// colour-blocked order (C = 3 on a nine-block finest level, 9 on a 21-block one, 2 on five-point
// levels); offsets in elements of the value type.
struct Level2D {
    int nx, ny, nb, pad;
    Perm2D P;
    long long J, Dinv, rhs, dU;
};

// ---- launchers (return hipError_t of the launch) ----------------------------------------

// residual over tiles (batched: tiles index instances) or one instance (tiles == null)
// recon: the reconstruction of every instance in the launch (NMG_RECON_*)
hipError_t launch_residual1d(const Inst1D *insts_dev, const Tile *tiles, int ntiles,
                             const Inst1D *single, NewtonState *state, double *partial, int recon,
                             hipStream_t s);
hipError_t launch_res_finalize(const Inst1D *insts_dev, int ninst, NewtonState *state,
                               const double *partial, int init, hipStream_t s);
hipError_t launch_sum_res(const double *rn, int N, double *res, hipStream_t s);
// Jacobian: writes FP64 (prec 0) or FP32 (prec 1) blocks with row stride N at J_out (single) or
// at each instance's level-0 J (batched, via the level table).  fused_partial (batched only):
// evaluate the residual in the same launch (the tiles' sums of ||R_j||_1 go to fused_partial,
// in the order of the tile list) instead of reading R and ||R_j||_1
hipError_t launch_jacobian1d(const Inst1D *insts_dev, const Tile *tiles, int ntiles,
                             const Inst1D *single, double *J_single, const MGArgs &mg, int prec,
                             int nb_mask, int recon, hipStream_t s, double *fused_partial = nullptr);
hipError_t launch_coarsen1d(const MGArgs &mg, const Tile *tiles, int ntiles, int prec, hipStream_t s);
// nt: threads of the bottom workgroup (256, 512 or 1024); it handles levels of up to 2 nt cells
hipError_t launch_bottom(const MGArgs &mg, const int *inst_list, int n, int zero_init0, int final_update,
                         int prec, int nt, hipStream_t s);
// mode 0: pre-smoothing + restriction; 1: prolongation + post-smoothing (+ update); 2: both,
// the post-smoothing of one V-cycle and the pre-smoothing of the next on one level.  src_out:
// read dU from dUo (1) or dU (0) and write the other buffer.
hipError_t launch_smooth1d(const MGArgs &mg, const Tile *tiles, int ntiles, int nb_mask, int mode,
                           int zero_init, int final_update, int src_out, int prec, int tile, int reverse, hipStream_t s);
hipError_t launch_convert(const void *src, int src_prec, void *dst, int dst_prec, long long n,
                          hipStream_t s);
// Newton-SOR (section 5.1.1) on level 0: one symmetric multicolour block-SOR step per launch
// with the per-tile l1 change of dU in partial[], the per-instance stopping test, the
// lexicographic variant (one thread per instance, test included) and the update U += tau dU
// Newton-SOR step `step` of a Newton step: reads dU (even steps) or dUo (odd), writes the other
hipError_t launch_sor_mc(const MGArgs &mg, const Tile *tiles, int ntiles, int nb_max, int step,
                         double *partial, int prec, hipStream_t s);
hipError_t launch_sor_finalize(const Inst1D *insts, int ninst, NewtonState *state, const double *partial,
                               double tol, hipStream_t s);
hipError_t launch_sor_lex(const MGArgs &mg, int ninst, int nb_max, int zero_init, double tol, int prec,
                          hipStream_t s);
// U += tau dU on level 0, dU taken from dUo when from_out
hipError_t launch_update1d(const MGArgs &mg, const Tile *tiles, int ntiles, int from_out, int prec, hipStream_t s);
// Appendix A interpolation of a 1D state [2][nc] to [2][2 nc]
hipError_t launch_interp_a2(const double *Uc, int nc, double *Uf, hipStream_t s);
// Appendix A interpolation of a 2D state [3][nyc][nxc] to [3][2 nyc][2 nxc] (eq. A.3)
hipError_t launch_interp_a3(const double *Uc, int nxc, int nyc, double *Uf, hipStream_t s);

// 2D
int residual2d_tiles(int Nx, int Ny);
hipError_t launch_residual2d(const Inst2D &I, double *partial, hipStream_t s);
hipError_t launch_res2d_finalize(const double *partial, int ntiles, long long ncells, double *res,
                                 hipStream_t s);
// J, rhs, Dinv written in the cell order P (make_perm2d(Nx, Ny, 1) for the natural order)
hipError_t launch_jacobian2d(const Inst2D &I, const Perm2D &P, void *J, void *rhs, void *Dinv, int prec,
                             hipStream_t s, int nb = 9);
hipError_t launch_coarsen2d(void *mg, const Level2D &Lf, const Level2D &Lc, int prec, hipStream_t s);
// `reps` consecutive passes of one colour (the same neighbour values), one launch
// sched: NMG_SCHED2D_* bits (the pass form and the streaming hints; results are the same)
hipError_t launch_smooth2d_pass(void *mg, const Level2D &L, int colour, int reps, double omega, int prec,
                               hipStream_t s, int sched = 0);
hipError_t launch_restrict2d(void *mg, const Level2D &Lf, const Level2D &Lc, int prec, hipStream_t s);
hipError_t launch_prolong2d(void *mg, const Level2D &Lf, const Level2D &Lc, int prec, hipStream_t s);
// coarsest level: LU factors with row permutation (M*M doubles then M ints, M = 3 cells) once
// per operator; the solve with them runs in launch_bottom2d
hipError_t launch_coarse_factor2d(void *mg, const Level2D &L, double *lu, int prec, hipStream_t s);
// the levels first..nlev-1 of a V-cycle (down to the coarsest solve and back) in one workgroup
// sweeps: the levels' smoother is the directional sweeps D1-D4 instead of the multicolour schedule
hipError_t launch_bottom2d(void *mg, const Level2D *levels, int first, int nlev, int nu1, int nu2, double omega,
                           const double *lu, int prec, hipStream_t s, int sweeps = 0);
// nu iterations of the directional sweeps D1-D4 on one level (one workgroup)
hipError_t launch_sweeps2d(void *mg, const Level2D &L, int nu, double omega, int prec, hipStream_t s);
constexpr long long kBottom2DCells = 512;    // levels at most this size go to launch_bottom2d
inline size_t coarse_lu_bytes(int M) { return sizeof(double) * (size_t)M * M + sizeof(int) * (size_t)M; }
hipError_t launch_fill(void *p, int prec, long long n, hipStream_t s);
hipError_t launch_update2d(double *U, const void *mg, const Level2D &L0, double tau,
                           const NewtonState *state, int prec, hipStream_t s);
hipError_t launch_dinv2d(const double *J, void *Dinv, const Level2D &L0, int prec, hipStream_t s);
// nent per-cell entries between the natural order (src or dst, per `to_level`) and a level's order
hipError_t launch_permute2d(const void *src, int src_prec, void *dst, int dst_prec, const Level2D &L, int nent,
                            int to_level, hipStream_t s);
hipError_t launch_state2d(const double *partial, int ntiles, long long ncells, double tol, int n_max,
                          NewtonState *state, double *hist, int max_hist, int init, hipStream_t s);
constexpr int kMaxCoarse2D = 40;   // cells on the coarsest 2D level (dense solve in LDS)

// error reporting shared by the host translation units (sets the thread-local message)
nmg_status set_error(nmg_status st, const char *msg);

// 2D entry points (dim = 2), called by the ABI functions
size_t workspace2d_bytes(const nmg_desc *d, const nmg_params *p);
nmg_status residual2d(const nmg_desc *d, const double *U, double *R, double *rn, double *res,
                      hipStream_t s);
nmg_status jacobian2d(const nmg_desc *d, const nmg_params *p, const double *U, const double *R,
                      const double *rn, double *J, hipStream_t s);
nmg_status vcycle2d(const nmg_desc *d, const nmg_params *p, void *ws, size_t ws_bytes, const void *J,
                    const void *rhs, void *dU, int setup, hipStream_t s);
nmg_status newton2d(const nmg_desc *d, const nmg_params *p, void *ws, size_t ws_bytes, double *U,
                    nmg_stats *stats, double *hist, int max_hist, hipStream_t s);
nmg_status newton2d_begin(const nmg_desc *d, const nmg_params *p, void *ws, size_t ws_bytes, double *U, hipStream_t s);
nmg_status autotune2d(const nmg_desc *d, const nmg_params *p, void *ws, size_t ws_bytes, const double *J,
                      const void *rhs, int cycles, int *best, double *ms, hipStream_t s);
nmg_status newton2d_steps(const nmg_desc *d, const nmg_params *p, void *ws, size_t ws_bytes, double *U, int steps,
                          nmg_newton_state *state_out, hipStream_t s);

}  // namespace nmg
