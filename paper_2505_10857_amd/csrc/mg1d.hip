// Geometric multigrid for the 1D regularised Newton systems (section 3.4, eq. 15-19,
// Algorithm 2) on gfx950.
//
//  * k_coarsen: coarse operators of eq. (17) for up to ten levels in one launch.  A workgroup
//    owns an aligned run of 1024 cells of the starting level and reduces them level by level
//    in LDS (each coarse cell aggregates two children, eq. 15), writing every level's blocks.
//    The smoothers form the closed-form 2x2 inverses of the diagonal blocks of eq. (19)
//    themselves, so no inverse is stored.
//  * k_smooth: all nu multicolour block-SOR half-sweeps of one smoothing phase fused in one
//    launch.  Each workgroup loads its cells' block rows and right-hand side into
//    registers once, keeps dU in LDS, and runs the half-sweeps with a halo wide enough that
//    the cells it writes are exact; the pre-smoothing kernel then forms the restricted
//    right-hand side of eq. (17), the post-smoothing kernel first adds the prolongation of
//    eq. (18) (and, at the finest level after the last cycle, applies the Newton update of
//    eq. 14).  HBM traffic per level and phase is one read of the operator.
//  * k_bottom: all small levels of one instance in one workgroup: smoothing and restriction
//    down, the coarsest system solved exactly (up to rounding) by block parallel cyclic
//    reduction, prolongation and smoothing back up.
#include "nmg_common.h"

namespace nmg {

template <typename T>
__device__ __forceinline__ double ld(const T *p, long long i) { return (double)p[i]; }

__device__ __forceinline__ bool active_of(const MGArgs &mg, int inst)
{
    return mg.state == nullptr || mg.state[mg.insts[inst].active_idx].active;
}

__device__ __forceinline__ void inv2(const double A[4], double B[4])
{
    double det = A[0] * A[3] - A[1] * A[2];
    B[0] = A[3] / det;
    B[1] = -A[1] / det;
    B[2] = -A[2] / det;
    B[3] = A[0] / det;
}

// ---- coarse operators --------------------------------------------------------------------

// Children blocks (b = 0..nb-1 <-> column offsets -nb/2..nb/2) of cells 2jc and 2jc+1 ->
// coarse tridiagonal row of cell jc, summing the fine blocks of eq. (17) in order of the
// child row and then the child column.
__device__ __forceinline__ void coarse_row(int nb, const double (*f0)[4], const double (*f1)[4],
                                           double Wc[4], double Dc[4], double Ec[4])
{
#pragma unroll
    for (int e = 0; e < 4; e++) {
        if (nb == 5) {
            Wc[e] = f0[0][e] + f0[1][e] + f1[0][e];
            Dc[e] = f0[2][e] + f0[3][e] + f1[1][e] + f1[2][e];
            Ec[e] = f0[4][e] + f1[3][e] + f1[4][e];
        } else {
            Wc[e] = f0[0][e];
            Dc[e] = f0[1][e] + f0[2][e] + f1[0][e] + f1[1][e];
            Ec[e] = f1[2][e];
        }
    }
}

template <typename T, int NB>
__device__ __forceinline__ void first_coarse(const Level1D &L0, const Level1D &Lc, T *base, int c0,
                                             int t, double (*blk)[12])
{
    for (int k = 0; k < kCoarsenCells / 2; k++) {
        const int jl = t * (kCoarsenCells / 2) + k;   // local coarse index
        const int jc = c0 + jl;
        if (jc >= Lc.n) break;
        double f0[5][4], f1[5][4];
#pragma unroll
        for (int b = 0; b < NB; b++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                f0[b][e] = ld(base + L0.J, (b * 4 + e) * (long long)L0.n + 2 * jc);
                f1[b][e] = ld(base + L0.J, (b * 4 + e) * (long long)L0.n + 2 * jc + 1);
            }
        double W[4], D[4], E[4];
        coarse_row(NB, f0, f1, W, D, E);
#pragma unroll
        for (int e = 0; e < 4; e++) {
            blk[jl][e] = W[e]; blk[jl][4 + e] = D[e]; blk[jl][8 + e] = E[e];
            base[Lc.J + (0 * 4 + e) * (long long)Lc.n + jc] = (T)W[e];
            base[Lc.J + (1 * 4 + e) * (long long)Lc.n + jc] = (T)D[e];
            base[Lc.J + (2 * 4 + e) * (long long)Lc.n + jc] = (T)E[e];
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kTile) k_coarsen(MGArgs mg, const Tile *tiles)
{
    constexpr int CPT = kCoarsenCells;           // level-l0 cells per thread
    constexpr int SPAN = kTile * CPT;             // level-l0 cells per workgroup
    __shared__ double blk[SPAN / 2][12];          // current coarse level: W, D, E per cell
    const Tile tl = tiles[blockIdx.x];
    const Level1D L0 = mg.levs[tl.lev];
    if (!active_of(mg, L0.inst)) return;
    T *base = reinterpret_cast<T *>(mg.mg);
    const int t = threadIdx.x;
    const int nb = L0.nb;

    if (L0.coarsest) return;

    // first coarse level from the starting level (global reads)
    int lev = L0.child;
    Level1D Lc = mg.levs[lev];
    const int c0 = tl.a / 2;                      // first coarse cell of this tile
    if (nb == 5) first_coarse<T, 5>(L0, Lc, base, c0, t, blk);
    else first_coarse<T, 3>(L0, Lc, base, c0, t, blk);
    __syncthreads();

    // further levels from LDS
    int cnt = SPAN / 2;     // cells of the current level held by this tile
    int cstart = c0;        // first cell (level index) of the current level in this tile
    while (!Lc.coarsest && cnt >= 2) {
        const int nlev = Lc.child;
        const Level1D Ln = mg.levs[nlev];
        const int nstart = cstart / 2;
        const int ncnt = cnt / 2;
        double W[4], D[4], E[4];
        const int jc = nstart + t;
        const bool mine = t < ncnt && jc < Ln.n;
        if (mine) {
            double f0[5][4], f1[5][4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                f0[0][e] = blk[2 * t][e]; f0[1][e] = blk[2 * t][4 + e]; f0[2][e] = blk[2 * t][8 + e];
                f1[0][e] = blk[2 * t + 1][e]; f1[1][e] = blk[2 * t + 1][4 + e]; f1[2][e] = blk[2 * t + 1][8 + e];
            }
            coarse_row(3, f0, f1, W, D, E);
        }
        __syncthreads();
        if (mine) {
            for (int e = 0; e < 4; e++) {
                blk[t][e] = W[e]; blk[t][4 + e] = D[e]; blk[t][8 + e] = E[e];
                base[Ln.J + (0 * 4 + e) * (long long)Ln.n + jc] = (T)W[e];
                base[Ln.J + (1 * 4 + e) * (long long)Ln.n + jc] = (T)D[e];
                base[Ln.J + (2 * 4 + e) * (long long)Ln.n + jc] = (T)E[e];
            }
        }
        __syncthreads();
        Lc = Ln;
        cnt = ncnt;
        cstart = nstart;
    }
}

// ---- fused smoother ------------------------------------------------------------------------

// mode 0: (zero or loaded) dU -> nu1 symmetric steps -> write dU, restrict rhs to the child.
// mode 1: dU + prolongated child dU -> nu2 symmetric steps -> write dU (or update U).
// mode 2: dU + prolongated child dU -> nu2 + nu1 symmetric steps (the post-smoothing of one
//         V-cycle and the pre-smoothing of the next, with nothing between them on this level)
//         -> write dU, restrict rhs to the child; its tiles have the wider halo halo2.
// src_out: the tile reads dU from dUo (1) or dU (0) and writes its cells to the other buffer.
template <typename T, int NB, int MODE, int TW>
__global__ void __launch_bounds__(TW) k_smooth(MGArgs mg, const Tile *tiles, int zero_init,
                                                  int final_update, int src_out, int reverse)
{
    constexpr int mode = MODE;
    constexpr int HW = NB / 2;
    constexpr int C = NB == 5 ? 3 : 2;
    __shared__ double s0[TW + 2 * HW], s1[TW + 2 * HW];
    // reverse: the last tiles first (workgroups start roughly in index order), so that a pass
    // that follows another pass over the same data begins with what that pass touched last,
    // which is still in the memory-side cache
    const Tile tl = tiles[reverse ? gridDim.x - 1 - blockIdx.x : blockIdx.x];
    const Level1D L = mg.levs[tl.lev];
    if (L.nb != NB) return;
    if (!active_of(mg, L.inst)) return;
    const Inst1D &I = mg.insts[L.inst];
    T *base = reinterpret_cast<T *>(mg.mg);
    const int n = L.n, h = mode == 2 ? L.halo2 : L.halo, V = mode == 2 ? L.V2 : L.V;
    const int t = threadIdx.x;
    const int j = tl.a - h + t;
    const bool in = j >= 0 && j < n;
    // the halo of a tile must hold the values from before the launch, so the cells are written
    // to the other buffer
    const long long src = src_out ? L.dUo : L.dU, dst = src_out ? L.dU : L.dUo;

    double Jr[NB][4], D[4], r0 = 0.0, r1 = 0.0, du0 = 0.0, du1 = 0.0;
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
        for (int e = 0; e < 4; e++) Jr[b][e] = in ? ld(base + L.J, (b * 4 + e) * (long long)n + j) : 0.0;
    // the inverse of the diagonal block, formed here instead of read (one division per cell
    // and launch against 4 values of HBM traffic per cell and half-sweep phase)
    if (in) inv2(Jr[HW], D);
    else D[0] = D[1] = D[2] = D[3] = 0.0;
    if (in) {
        r0 = ld(base + L.rhs, j);
        r1 = ld(base + L.rhs, n + (long long)j);
        if (!(mode == 0 && zero_init)) {
            du0 = ld(base + src, j);
            du1 = ld(base + src, n + (long long)j);
        }
        if (mode != 0) {
            const Level1D &Lc = mg.levs[L.child];
            du0 = du0 + ld(base + Lc.dU, j >> 1);
            du1 = du1 + ld(base + Lc.dU, Lc.n + (long long)(j >> 1));
        }
    }
    s0[t + HW] = du0;
    s1[t + HW] = du1;
    if (t < HW) { s0[t] = 0.0; s1[t] = 0.0; s0[TW + HW + t] = 0.0; s1[TW + HW + t] = 0.0; }
    __syncthreads();

    const double w = I.omega;
    const int col = ((j % C) + C) % C;
    // mode 2 runs the post-smoothing steps, rounds dU to the storage type as the separate
    // launches would when storing it, then the pre-smoothing steps
    for (int phase = 0; phase < (mode == 2 ? 2 : 1); phase++) {
        const int steps = mode == 0 ? I.nu1 : mode == 1 ? I.nu2 : phase == 0 ? I.nu2 : I.nu1;
        if (phase == 1) {
            du0 = (double)(T)du0;
            du1 = (double)(T)du1;
            s0[t + HW] = du0;
            s1[t + HW] = du1;
            __syncthreads();
        }
        // half-sweep colours 0..C-1, C-1..0 per step; a run of equal colours (at every turn)
        // sees the same neighbour values, so its relaxations share one off-diagonal sum
        const int total = steps * 2 * C;
        int cur = -1, reps = 0;
        for (int q = 0; q <= total; q++) {
            const int hs = q % (2 * C);
            const int c = q == total ? -1 : (hs < C ? hs : 2 * C - 1 - hs);
            if (c == cur) { reps++; continue; }
            if (reps > 0) {
                if (in && col == cur) {
                    // eq. (19): dU_j <- (1-w) dU_j - w J_jj^{-1} (rhs_j + sum_{i != j} J_ji dU_i)
                    double a0 = r0, a1 = r1;
#pragma unroll
                    for (int b = 0; b < NB; b++) {
                        if (b == HW) continue;
                        const double x0 = s0[t + b], x1 = s1[t + b];
                        a0 = a0 + (Jr[b][0] * x0 + Jr[b][1] * x1);
                        a1 = a1 + (Jr[b][2] * x0 + Jr[b][3] * x1);
                    }
                    const double t0 = D[0] * a0 + D[1] * a1;
                    const double t1 = D[2] * a0 + D[3] * a1;
                    for (int k = 0; k < reps; k++) {
                        du0 = (1.0 - w) * du0 - w * t0;
                        du1 = (1.0 - w) * du1 - w * t1;
                    }
                    s0[t + HW] = du0;
                    s1[t + HW] = du1;
                }
                __syncthreads();
            }
            cur = c;
            reps = 1;
        }
    }

    const bool valid = in && t >= h && t < h + V;
    if (mode != 1) {
        // restriction, eq. (17): rhs_c = sum over the two children of (rhs + sum_i J dU_i)
        double a0 = r0, a1 = r1;
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const double x0 = s0[t + b], x1 = s1[t + b];
            a0 = a0 + (Jr[b][0] * x0 + Jr[b][1] * x1);
            a1 = a1 + (Jr[b][2] * x0 + Jr[b][3] * x1);
        }
        const double p0 = __shfl_xor(a0, 1, 64);
        const double p1 = __shfl_xor(a1, 1, 64);
        if (valid) {
            base[dst + j] = (T)du0;
            base[dst + n + (long long)j] = (T)du1;
            if ((j & 1) == 0 && !L.coarsest) {
                const Level1D &Lc = mg.levs[L.child];
                base[Lc.rhs + (j >> 1)] = (T)(a0 + p0);
                base[Lc.rhs + Lc.n + (long long)(j >> 1)] = (T)(a1 + p1);
            }
        }
    } else if (valid) {
        if (final_update) {
            // eq. (14): U <- U + tau dU
            I.U[j] = I.U[j] + I.tau * du0;
            I.U[I.N + j] = I.U[I.N + j] + I.tau * du1;
        } else {
            base[dst + j] = (T)du0;
            base[dst + n + (long long)j] = (T)du1;
        }
    }
}

// ---- coarsest level ------------------------------------------------------------------------
// The coarsest system  W_j x_{j-1} + D_j x_j + E_j x_{j+1} = -rhs_j  (2x2 blocks) is solved
// exactly by block parallel cyclic reduction: step k (stride s = 2^k) eliminates the couplings
// at distance s from every row at once,
//     a_j = -W_j D_{j-s}^{-1},  g_j = -E_j D_{j+s}^{-1},
//     W_j <- a_j W_{j-s},  E_j <- g_j E_{j+s},  D_j <- D_j + a_j E_{j-s} + g_j W_{j+s},
// and the same combination of right-hand sides; after ceil(log2 n) steps every row is
// decoupled and x_j = D_j^{-1} b_j.  One thread per cell, 2x2 blocks in LDS, inside the
// bottom-of-cycle kernel below.

__device__ __forceinline__ void mul2(const double A[4], const double B[4], double C[4])
{
    C[0] = A[0] * B[0] + A[1] * B[2];
    C[1] = A[0] * B[1] + A[1] * B[3];
    C[2] = A[2] * B[0] + A[3] * B[2];
    C[3] = A[2] * B[1] + A[3] * B[3];
}

// ---- bottom of the V-cycle -----------------------------------------------------------------
// Every level with at most 2 NT cells (always including the coarsest; the plan picks the first
// such level) is handled by one NT-thread workgroup per instance in a single launch:
// pre-smoothing and restriction down to the coarsest level, the cyclic-reduction solve there,
// prolongation and post-smoothing back up.  Thread t owns cells t and t + NT of every level;
// dU of the current level lives in LDS,
// the restricted right-hand sides of all levels below the first stay in LDS, and the
// pre-smoothed dU of each level goes to HBM and comes back to the thread that wrote it.
// Same arithmetic, in the same order, as the per-level kernels.

template <typename T>
__device__ __forceinline__ void bottom_load(const T *base, const Level1D &L, int c, double Jr[12], double D[4])
{
#pragma unroll
    for (int e = 0; e < 12; e++) Jr[e] = ld(base + L.J, e * (long long)L.n + c);
    inv2(&Jr[4], D);   // the inverse of the diagonal block, as in the tiled smoother
}

template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_bottom(MGArgs mg, const int *inst_list, int zero_init0,
                                               int final_update)
{
    static_assert(2 * NT >= kMaxCoarse, "the coarsest level needs one thread per cell");
    __shared__ double u0[2 * NT + 2], u1[2 * NT + 2];   // dU of the current level, index c+1
    __shared__ double q0[2 * NT], q1[2 * NT];           // rhs of the levels below the first
    __shared__ double sW[kMaxCoarse][4], sD[kMaxCoarse][4], sE[kMaxCoarse][4], sDi[kMaxCoarse][4];
    const int inst = inst_list[blockIdx.x];
    if (!active_of(mg, inst)) return;
    const Inst1D &I = mg.insts[inst];
    T *base = reinterpret_cast<T *>(mg.mg);
    const int t = threadIdx.x;
    const int lb = I.lev0 + I.lbot;           // level-table index of the first bottom level
    const double w = I.omega;
    if (t == 0) { u0[0] = u1[0] = 0.0; }
    {   // the coarsest operator, staged once (read at the end of the descent)
        const Level1D Lc = mg.levs[I.levc];
        if (t < Lc.n) {
#pragma unroll
            for (int e = 0; e < 4; e++) {
                sW[t][e] = ld(base + Lc.J, (0 * 4 + e) * (long long)Lc.n + t);
                sD[t][e] = ld(base + Lc.J, (1 * 4 + e) * (long long)Lc.n + t);
                sE[t][e] = ld(base + Lc.J, (2 * 4 + e) * (long long)Lc.n + t);
            }
        }
    }

    // ---- down: pre-smoothing and restriction -------------------------------------------
    int li = lb, qoff = 0;                    // qoff: LDS offset of this level's rhs (levels > lb)
    while (true) {
        const Level1D L = mg.levs[li];
        if (L.coarsest) break;
        const int n = L.n;
        double Jr[2][12], D[2][4], r[2][2], du[2][2];
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int c = t + k * NT;
            du[k][0] = du[k][1] = 0.0;
            r[k][0] = r[k][1] = 0.0;
            if (c < n) {
                bottom_load(base, L, c, Jr[k], D[k]);
                if (li == lb) {
                    r[k][0] = ld(base + L.rhs, c);
                    r[k][1] = ld(base + L.rhs, n + (long long)c);
                    if (li == I.lev0 && !zero_init0) {
                        du[k][0] = ld(base + L.dU, c);
                        du[k][1] = ld(base + L.dU, n + (long long)c);
                    }
                } else {
                    r[k][0] = q0[qoff + c];
                    r[k][1] = q1[qoff + c];
                }
                u0[c + 1] = du[k][0];
                u1[c + 1] = du[k][1];
            }
        }
        if (t == 0) { u0[n + 1] = 0.0; u1[n + 1] = 0.0; }
        __syncthreads();
        // half-sweeps 0 1 1 0 per step: runs 0, (1 1), (0 0), ..., (1 1), 0 of one colour
        // share the neighbour values and so one off-diagonal sum
        for (int run = 0; I.nu1 > 0 && run <= 2 * I.nu1; run++) {
            const int col = run & 1, reps = (run == 0 || run == 2 * I.nu1) ? 1 : 2;
#pragma unroll
            for (int k = 0; k < 2; k++) {
                const int c = t + k * NT;
                if (c < n && (c & 1) == col) {
                    const double x0 = u0[c], x1 = u1[c], y0 = u0[c + 2], y1 = u1[c + 2];
                    double a0 = r[k][0], a1 = r[k][1];
                    a0 = a0 + (Jr[k][0] * x0 + Jr[k][1] * x1);
                    a1 = a1 + (Jr[k][2] * x0 + Jr[k][3] * x1);
                    a0 = a0 + (Jr[k][8] * y0 + Jr[k][9] * y1);
                    a1 = a1 + (Jr[k][10] * y0 + Jr[k][11] * y1);
                    const double t0 = D[k][0] * a0 + D[k][1] * a1;
                    const double t1 = D[k][2] * a0 + D[k][3] * a1;
                    for (int q = 0; q < reps; q++) {
                        du[k][0] = (1.0 - w) * du[k][0] - w * t0;
                        du[k][1] = (1.0 - w) * du[k][1] - w * t1;
                    }
                    u0[c + 1] = du[k][0];
                    u1[c + 1] = du[k][1];
                }
            }
            __syncthreads();
        }
        // restriction to the child (eq. 17) into LDS; pre-smoothed dU to HBM
        const int qn = li == lb ? 0 : qoff + n;
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int c = t + k * NT;
            double a0 = r[k][0], a1 = r[k][1];
            if (c < n) {
                const double x0 = u0[c], x1 = u1[c], y0 = u0[c + 2], y1 = u1[c + 2];
                a0 = a0 + (Jr[k][0] * x0 + Jr[k][1] * x1);
                a1 = a1 + (Jr[k][2] * x0 + Jr[k][3] * x1);
                a0 = a0 + (Jr[k][4] * du[k][0] + Jr[k][5] * du[k][1]);
                a1 = a1 + (Jr[k][6] * du[k][0] + Jr[k][7] * du[k][1]);
                a0 = a0 + (Jr[k][8] * y0 + Jr[k][9] * y1);
                a1 = a1 + (Jr[k][10] * y0 + Jr[k][11] * y1);
            }
            const double p0 = __shfl_xor(a0, 1, 64), p1 = __shfl_xor(a1, 1, 64);
            if (c < n) {
                // rounded to the value type as the tiled kernels round it in HBM, so the result
                // does not depend on which levels run here
                if ((c & 1) == 0) {
                    q0[qn + (c >> 1)] = (double)(T)(a0 + p0);
                    q1[qn + (c >> 1)] = (double)(T)(a1 + p1);
                }
                base[L.dU + c] = (T)du[k][0];
                base[L.dU + n + (long long)c] = (T)du[k][1];
            }
        }
        __syncthreads();
        qoff = qn;
        li = L.child;
    }

    // ---- coarsest: block parallel cyclic reduction on the staged operator ---------------------
    {
        const Level1D L = mg.levs[li];
        const int n = L.n;
        double W[4] = {0, 0, 0, 0}, Dm[4] = {1, 0, 0, 1}, E[4] = {0, 0, 0, 0};
        double b0 = 0.0, b1 = 0.0;
        if (t < n) {
#pragma unroll
            for (int e = 0; e < 4; e++) { W[e] = sW[t][e]; Dm[e] = sD[t][e]; E[e] = sE[t][e]; }
            if (li == lb) { b0 = -ld(base + L.rhs, t); b1 = -ld(base + L.rhs, n + (long long)t); }
            else { b0 = -q0[qoff + t]; b1 = -q1[qoff + t]; }
        }
        for (int st = 1; st < n; st <<= 1) {
            double Di[4];
            inv2(Dm, Di);
            __syncthreads();
            if (t < n) {
#pragma unroll
                for (int e = 0; e < 4; e++) { sW[t][e] = W[e]; sD[t][e] = Dm[e]; sE[t][e] = E[e]; sDi[t][e] = Di[e]; }
                u0[t + 1] = b0;
                u1[t + 1] = b1;
            }
            __syncthreads();
            if (t < n) {
                double Wn[4] = {0, 0, 0, 0}, En[4] = {0, 0, 0, 0}, Dn[4], a[4], g[4], tm[4];
#pragma unroll
                for (int e = 0; e < 4; e++) Dn[e] = Dm[e];
                double bn0 = b0, bn1 = b1;
                if (t - st >= 0) {
                    mul2(W, sDi[t - st], tm);
#pragma unroll
                    for (int e = 0; e < 4; e++) a[e] = -tm[e];
                    mul2(a, sW[t - st], Wn);
                    mul2(a, sE[t - st], tm);
#pragma unroll
                    for (int e = 0; e < 4; e++) Dn[e] = Dn[e] + tm[e];
                    const double c0 = u0[t - st + 1], c1 = u1[t - st + 1];
                    bn0 = bn0 + (a[0] * c0 + a[1] * c1);
                    bn1 = bn1 + (a[2] * c0 + a[3] * c1);
                }
                if (t + st < n) {
                    mul2(E, sDi[t + st], tm);
#pragma unroll
                    for (int e = 0; e < 4; e++) g[e] = -tm[e];
                    mul2(g, sE[t + st], En);
                    mul2(g, sW[t + st], tm);
#pragma unroll
                    for (int e = 0; e < 4; e++) Dn[e] = Dn[e] + tm[e];
                    const double c0 = u0[t + st + 1], c1 = u1[t + st + 1];
                    bn0 = bn0 + (g[0] * c0 + g[1] * c1);
                    bn1 = bn1 + (g[2] * c0 + g[3] * c1);
                }
#pragma unroll
                for (int e = 0; e < 4; e++) { W[e] = Wn[e]; E[e] = En[e]; Dm[e] = Dn[e]; }
                b0 = bn0;
                b1 = bn1;
            }
        }
        __syncthreads();
        if (t < n) {
            double Di[4];
            inv2(Dm, Di);
            const double x0 = Di[0] * b0 + Di[1] * b1;
            const double x1 = Di[2] * b0 + Di[3] * b1;
            u0[t + 1] = x0;
            u1[t + 1] = x1;
            if (li == I.lev0 && final_update) {   // one-level hierarchy: the Newton update, eq. (14)
                I.U[t] = I.U[t] + I.tau * x0;
                I.U[I.N + t] = I.U[I.N + t] + I.tau * x1;
            } else if (li == lb) {   // the bottom is the coarsest level only
                base[L.dU + t] = (T)x0;
                base[L.dU + n + (long long)t] = (T)x1;
            }
        }
        __syncthreads();
    }

    // ---- up: prolongation and post-smoothing ------------------------------------------------
    while (li > lb) {
        li -= 1;
        const Level1D L = mg.levs[li];
        const int n = L.n;
        // rhs offset of this level: walk the offsets again (levels above lb only)
        int qo = 0;
        for (int x = lb + 1; x < li; x++) qo += mg.levs[x].n;
        double par[2][2];
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int c = t + k * NT;
            par[k][0] = par[k][1] = 0.0;
            if (c < n) { par[k][0] = (double)(T)u0[(c >> 1) + 1]; par[k][1] = (double)(T)u1[(c >> 1) + 1]; }
        }
        __syncthreads();
        double Jr[2][12], D[2][4], r[2][2], du[2][2];
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int c = t + k * NT;
            du[k][0] = du[k][1] = 0.0;
            r[k][0] = r[k][1] = 0.0;
            if (c < n) {
                bottom_load(base, L, c, Jr[k], D[k]);
                if (li == lb) {
                    r[k][0] = ld(base + L.rhs, c);
                    r[k][1] = ld(base + L.rhs, n + (long long)c);
                } else {
                    r[k][0] = q0[qo + c];
                    r[k][1] = q1[qo + c];
                }
                du[k][0] = ld(base + L.dU, c) + par[k][0];
                du[k][1] = ld(base + L.dU, n + (long long)c) + par[k][1];
                u0[c + 1] = du[k][0];
                u1[c + 1] = du[k][1];
            }
        }
        if (t == 0) { u0[n + 1] = 0.0; u1[n + 1] = 0.0; }
        __syncthreads();
        // half-sweeps 0 1 1 0 per step: runs 0, (1 1), (0 0), ..., (1 1), 0 of one colour
        // share the neighbour values and so one off-diagonal sum
        for (int run = 0; I.nu2 > 0 && run <= 2 * I.nu2; run++) {
            const int col = run & 1, reps = (run == 0 || run == 2 * I.nu2) ? 1 : 2;
#pragma unroll
            for (int k = 0; k < 2; k++) {
                const int c = t + k * NT;
                if (c < n && (c & 1) == col) {
                    const double x0 = u0[c], x1 = u1[c], y0 = u0[c + 2], y1 = u1[c + 2];
                    double a0 = r[k][0], a1 = r[k][1];
                    a0 = a0 + (Jr[k][0] * x0 + Jr[k][1] * x1);
                    a1 = a1 + (Jr[k][2] * x0 + Jr[k][3] * x1);
                    a0 = a0 + (Jr[k][8] * y0 + Jr[k][9] * y1);
                    a1 = a1 + (Jr[k][10] * y0 + Jr[k][11] * y1);
                    const double t0 = D[k][0] * a0 + D[k][1] * a1;
                    const double t1 = D[k][2] * a0 + D[k][3] * a1;
                    for (int q = 0; q < reps; q++) {
                        du[k][0] = (1.0 - w) * du[k][0] - w * t0;
                        du[k][1] = (1.0 - w) * du[k][1] - w * t1;
                    }
                    u0[c + 1] = du[k][0];
                    u1[c + 1] = du[k][1];
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < 2; k++) {
            const int c = t + k * NT;
            if (c >= n) continue;
            if (li == I.lev0 && final_update) {
                I.U[c] = I.U[c] + I.tau * du[k][0];
                I.U[I.N + c] = I.U[I.N + c] + I.tau * du[k][1];
            } else if (li == lb) {
                base[L.dU + c] = (T)du[k][0];
                base[L.dU + n + (long long)c] = (T)du[k][1];
            }
        }
    }
}

// ---- Newton-SOR (section 5.1.1) ----------------------------------------------------------
// The reference solver of the paper's Table 2: each Newton step solves the regularised system on
// the grid itself by symmetric block SOR steps (eq. 19) until the l1 norm of the change of dU
// between two successive steps falls below a tolerance or a step limit is reached.  The
// multicolour step reuses the tiled smoother's structure (one symmetric step per launch, halo
// for one step) and reports the change per tile; a finalisation launch per Newton-SOR step sums
// it per instance (fixed order) and marks the instance done, after which the later steps of the
// same Newton step skip it.

template <typename T, int NB>
__global__ void __launch_bounds__(kTile) k_sor_mc(MGArgs mg, const Tile *tiles, int step, double *partial)
{
    const bool zero_init = step == 0;
    constexpr int HW = NB / 2;
    constexpr int C = NB == 5 ? 3 : 2;
    __shared__ double s0[kTile + 2 * HW], s1[kTile + 2 * HW];
    __shared__ double red[kTile / 64];
    const Tile tl = tiles[blockIdx.x];
    const Level1D L = mg.levs[tl.lev];
    const int t = threadIdx.x;
    if (L.nb != NB) return;
    const Inst1D &I = mg.insts[L.inst];
    const NewtonState *S = mg.state ? &mg.state[I.active_idx] : nullptr;
    T *base = reinterpret_cast<T *>(mg.mg);
    const int n = L.n, h = L.halo;
    const int j = tl.a - h + t;
    const bool in = j >= 0 && j < n;
    // step k reads dU (k even) or dUo (k odd) and writes the other buffer
    const long long src = (step & 1) ? L.dUo : L.dU, dst = (step & 1) ? L.dU : L.dUo;
    if (S && (!S->active || S->sor_done)) {
        // stopped: carry the iterate over to the buffer the next step reads
        if (S->active && !zero_init && in && t >= h && t < h + L.V) {
            base[dst + j] = base[src + j];
            base[dst + n + (long long)j] = base[src + n + (long long)j];
        }
        if (t == 0) partial[blockIdx.x] = 0.0;
        return;
    }
    double Jr[NB][4], D[4], r0 = 0.0, r1 = 0.0, du0 = 0.0, du1 = 0.0;
#pragma unroll
    for (int b = 0; b < NB; b++)
#pragma unroll
        for (int e = 0; e < 4; e++) Jr[b][e] = in ? ld(base + L.J, (b * 4 + e) * (long long)n + j) : 0.0;
    if (in) inv2(Jr[HW], D);
    else D[0] = D[1] = D[2] = D[3] = 0.0;
    if (in) {
        r0 = ld(base + L.rhs, j);
        r1 = ld(base + L.rhs, n + (long long)j);
        if (!zero_init) {
            du0 = ld(base + src, j);
            du1 = ld(base + src, n + (long long)j);
        }
    }
    const double old0 = du0, old1 = du1;
    s0[t + HW] = du0;
    s1[t + HW] = du1;
    if (t < HW) { s0[t] = 0.0; s1[t] = 0.0; s0[kTile + HW + t] = 0.0; s1[kTile + HW + t] = 0.0; }
    __syncthreads();
    const double w = I.omega;
    const int col = ((j % C) + C) % C;
    for (int hs = 0; hs < 2 * C; hs++) {
        const int c = hs < C ? hs : 2 * C - 1 - hs;
        if (in && col == c) {
            double a0 = r0, a1 = r1;
#pragma unroll
            for (int b = 0; b < NB; b++) {
                if (b == HW) continue;
                const double x0 = s0[t + b], x1 = s1[t + b];
                a0 = a0 + (Jr[b][0] * x0 + Jr[b][1] * x1);
                a1 = a1 + (Jr[b][2] * x0 + Jr[b][3] * x1);
            }
            const double t0 = D[0] * a0 + D[1] * a1;
            const double t1 = D[2] * a0 + D[3] * a1;
            du0 = (1.0 - w) * du0 - w * t0;
            du1 = (1.0 - w) * du1 - w * t1;
            s0[t + HW] = du0;
            s1[t + HW] = du1;
        }
        __syncthreads();
    }
    const bool valid = in && t >= h && t < h + L.V;
    double v = 0.0;
    if (valid) {
        base[dst + j] = (T)du0;
        base[dst + n + (long long)j] = (T)du1;
        v = fabs((double)(T)du0 - old0) + fabs((double)(T)du1 - old1);
    }
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    if (t == 0) {
        double sum = 0.0;
        for (int k = 0; k < kTile / 64; k++) sum += red[k];
        partial[blockIdx.x] = sum;
    }
}

// per instance: the change of this Newton-SOR step from its tiles' partial sums
__global__ void __launch_bounds__(64) k_sor_finalize(const Inst1D *insts, int ninst, NewtonState *state,
                                                     const double *partial, double tol)
{
    const int b = blockIdx.x;
    if (b >= ninst) return;
    const Inst1D &I = insts[b];
    NewtonState &S = state[I.active_idx];
    if (!S.active || S.sor_done) return;
    double v = 0.0;
    for (int k = threadIdx.x; k < I.sor_tiles; k += 64) v += partial[I.sor_tile0 + k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (threadIdx.x == 0 && v < tol) S.sor_done = 1;
}

// The lexicographic symmetric step (forward then backward sweep, eq. 19) of one instance per
// workgroup, with its own stopping test.  The sweep is sequential (a cell uses the new values of
// the cells before it), so one lane performs it, reading from LDS: the workgroup stages it in
// chunks of kLexChunk cells in sweep order (the off-diagonal blocks, the inverse of the diagonal
// block -- formed by the loading lanes, not on the sweep's critical path -- the right-hand side
// and the current dU, plus the dU of HW cells ahead), three wavefronts loading the next chunk
// into the other buffer while the first lane sweeps the current one.  The sweeping lane keeps
// the new dU of the last HW cells in registers (the cells behind the next one, also across a
// chunk edge), and each swept chunk is written back before its buffer is refilled.  The change
// norm is summed in cell order by one lane from per-cell terms formed in parallel.  Every value
// and every sum is formed as the sequential sweep over global memory forms it, so the results
// are the same bit for bit.
constexpr int kLexChunk = 256;

template <typename T, int NB>
__device__ __forceinline__ void lex_load_chunk(const T *base, const Level1D &L, int n, int k, bool fwd, int t0,
                                               int nt, double (*bJ)[kLexChunk + NB - 1],
                                               double (*bR)[kLexChunk + NB - 1], double (*bU)[kLexChunk + NB - 1])
{
    constexpr int HW = NB / 2;
    for (int sl = HW + t0; sl < kLexChunk + 2 * HW; sl += nt) {   // the chunk and HW cells ahead
        const int q = k * kLexChunk - HW + sl;
        if (q >= n) continue;
        const int j = fwd ? q : n - 1 - q;
        bU[0][sl] = ld(base + L.dU, j);
        bU[1][sl] = ld(base + L.dU, n + (long long)j);
        if (sl < HW + kLexChunk) {
            bR[0][sl] = ld(base + L.rhs, j);
            bR[1][sl] = ld(base + L.rhs, n + (long long)j);
            double Jd[4], D[4];
#pragma unroll
            for (int e = 0; e < NB * 4; e++) {
                const double v = ld(base + L.J, e * (long long)n + j);
                if (e >= HW * 4 && e < HW * 4 + 4) Jd[e - HW * 4] = v;
                else bJ[e][sl] = v;
            }
            inv2(Jd, D);   // the diagonal block's slots hold its inverse
#pragma unroll
            for (int e = 0; e < 4; e++) bJ[HW * 4 + e][sl] = D[e];
        }
    }
}

template <typename T, int NB>
__global__ void __launch_bounds__(256) k_sor_lex(MGArgs mg, int zero_init, double tol)
{
    constexpr int HW = NB / 2, SL = kLexChunk + 2 * HW;
    __shared__ double bJ[2][NB * 4][SL], bR[2][2][SL], bU[2][2][SL];
    const Inst1D &I = mg.insts[blockIdx.x];
    NewtonState *S = mg.state ? &mg.state[I.active_idx] : nullptr;
    if (S && (!S->active || S->sor_done)) return;
    const Level1D L = mg.levs[I.lev0];
    if (L.nb != NB) return;
    T *base = reinterpret_cast<T *>(mg.mg);
    const int n = L.n, t = threadIdx.x;
    const double w = I.omega;
    // keep the iterate before this step in aux (zero at the first step of a Newton step)
    for (int j = t; j < n; j += blockDim.x) {
        const double d0 = zero_init ? 0.0 : ld(base + L.dU, j);
        const double d1 = zero_init ? 0.0 : ld(base + L.dU, n + (long long)j);
        base[L.aux + j] = (T)d0;
        base[L.aux + n + (long long)j] = (T)d1;
        if (zero_init) { base[L.dU + j] = (T)0.0; base[L.dU + n + (long long)j] = (T)0.0; }
    }
    __syncthreads();
    const int nch = (n + kLexChunk - 1) / kLexChunk;
    for (int pass = 0; pass < 2; pass++) {
        const bool fwd = pass == 0;
        lex_load_chunk<T, NB>(base, L, n, 0, fwd, t, blockDim.x, bJ[0], bR[0], bU[0]);
        __syncthreads();
        // lane 0: the new dU of the last HW cells swept, p[m] at m + 1 positions behind the next
        double p0[HW], p1[HW];
#pragma unroll
        for (int m = 0; m < HW; m++) p0[m] = p1[m] = 0.0;
        for (int k = 0; k < nch; k++) {
            const int b = k & 1;
            if (t == 0) {
                const int q1 = min(n, (k + 1) * kLexChunk);
                // unrolled: the loads of the next cells issue while this cell's chain runs
#pragma unroll 4
                for (int q = k * kLexChunk; q < q1; q++) {
                    const int j = fwd ? q : n - 1 - q;
                    const int sl = q - k * kLexChunk + HW;
                    double a0 = bR[b][0][sl], a1 = bR[b][1][sl];
#pragma unroll
                    for (int bb = 0; bb < NB; bb++) {
                        const int i = j + bb - HW;
                        if (bb == HW || i < 0 || i >= n) continue;
                        const int off = fwd ? bb - HW : HW - bb;   // position of cell i relative to q
                        double x0, x1;
                        if (off < 0) { x0 = p0[-off - 1]; x1 = p1[-off - 1]; }   // swept: its new value
                        else { x0 = bU[b][0][sl + off]; x1 = bU[b][1][sl + off]; }
                        a0 = a0 + (bJ[b][bb * 4 + 0][sl] * x0 + bJ[b][bb * 4 + 1][sl] * x1);
                        a1 = a1 + (bJ[b][bb * 4 + 2][sl] * x0 + bJ[b][bb * 4 + 3][sl] * x1);
                    }
                    const double D0 = bJ[b][HW * 4 + 0][sl], D1 = bJ[b][HW * 4 + 1][sl];
                    const double D2 = bJ[b][HW * 4 + 2][sl], D3 = bJ[b][HW * 4 + 3][sl];
                    const double t0 = D0 * a0 + D1 * a1;
                    const double t1 = D2 * a0 + D3 * a1;
                    const double d0 = bU[b][0][sl], d1 = bU[b][1][sl];
                    // rounded to the storage type, as the value a sweep over global memory reads back
                    const double n0 = (double)(T)((1.0 - w) * d0 - w * t0);
                    const double n1 = (double)(T)((1.0 - w) * d1 - w * t1);
                    bU[b][0][sl] = n0;
                    bU[b][1][sl] = n1;
#pragma unroll
                    for (int m = HW - 1; m > 0; m--) { p0[m] = p0[m - 1]; p1[m] = p1[m - 1]; }
                    p0[0] = n0;
                    p1[0] = n1;
                }
            } else if (t >= 64 && k + 1 < nch) {
                lex_load_chunk<T, NB>(base, L, n, k + 1, fwd, t - 64, blockDim.x - 64, bJ[b ^ 1], bR[b ^ 1], bU[b ^ 1]);
            }
            __syncthreads();
            for (int sl = HW + t; sl < HW + kLexChunk; sl += blockDim.x) {   // write the swept chunk back
                const int q = k * kLexChunk - HW + sl;
                if (q >= n) continue;
                const int j = fwd ? q : n - 1 - q;
                base[L.dU + j] = (T)bU[b][0][sl];
                base[L.dU + n + (long long)j] = (T)bU[b][1][sl];
            }
            __syncthreads();
        }
    }
    // l1 norm of the change over the whole step, cells in order, components interleaved
    double v = 0.0;
    for (int k = 0; k < nch; k++) {
        for (int c = t; c < kLexChunk; c += blockDim.x) {
            const int j = k * kLexChunk + c;
            if (j < n) {
                bR[0][0][c] = fabs(ld(base + L.dU, j) - ld(base + L.aux, j));
                bR[0][1][c] = fabs(ld(base + L.dU, n + (long long)j) - ld(base + L.aux, n + (long long)j));
            }
        }
        __syncthreads();
        if (t == 0) {
            const int c1 = min(kLexChunk, n - k * kLexChunk);
            for (int c = 0; c < c1; c++) {
                v += bR[0][0][c];
                v += bR[0][1][c];
            }
        }
        __syncthreads();
    }
    if (t == 0 && S && v < tol) S->sor_done = 1;
}

// eq. (14) after the Newton-SOR steps: U <- U + tau dU on level 0 of every active instance
template <typename T>
__global__ void __launch_bounds__(kTile) k_update1d(MGArgs mg, const Tile *tiles, int from_out)
{
    const Tile tl = tiles[blockIdx.x];
    const Inst1D &I = mg.insts[tl.lev];
    if (mg.state && !mg.state[I.active_idx].active) return;
    const Level1D L = mg.levs[I.lev0];
    const T *base = reinterpret_cast<const T *>(mg.mg);
    const int j = tl.a + threadIdx.x;
    if (j >= I.N) return;
    const long long d = from_out ? L.dUo : L.dU;
    I.U[j] = I.U[j] + I.tau * ld(base + d, j);
    I.U[I.N + j] = I.U[I.N + j] + I.tau * ld(base + d, L.n + (long long)j);
}

// Initial cell averages of a grid from the solution on the grid with half as many cells
// (Appendix A, eq. A.1-A.2), both components; one thread per coarse cell.  Interior cells use
// eq. (A.2); the first and last coarse cells average, over their two halves, the quadratic
// (A.1) of the neighbouring interior cell.
__global__ void k_interp_a2(const double *Uc, int nc, double *Uf)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= nc) return;
    const double *u = Uc + (long long)c * nc;
    double *v = Uf + (long long)c * 2 * nc;
    if (j >= 1 && j <= nc - 2) {
        v[2 * j] = u[j - 1] / 8.0 + u[j] - u[j + 1] / 8.0;
        v[2 * j + 1] = -u[j - 1] / 8.0 + u[j] + u[j + 1] / 8.0;
        return;
    }
    const int k = j == 0 ? 1 : nc - 2;          // centre of the quadratic used
    const double a = (u[k + 1] - u[k - 1]) / 2.0;
    const double b = (u[k - 1] - 2.0 * u[k] + u[k + 1]) / 2.0;
#pragma unroll
    for (int half = 0; half < 2; half++) {
        // this half of cell j spans xi in [lo, hi], xi = (x - x_k) / dx of the coarse grid
        const double lo = (double)(j - k) - 0.5 + 0.5 * half, hi = lo + 0.5;
        const double m1 = (lo + hi) / 2.0;
        const double m2 = (lo * lo + lo * hi + hi * hi) / 3.0;
        v[2 * j + half] = u[k] + a * m1 + b * (m2 - 1.0 / 12.0);
    }
}

hipError_t launch_sor_mc(const MGArgs &mg, const Tile *tiles, int ntiles, int nb_max, int step,
                         double *partial, int prec, hipStream_t s)
{
    if (ntiles == 0) return hipSuccess;
    if (prec == NMG_FP32_MG) {
        hipLaunchKernelGGL((k_sor_mc<float, 3>), dim3(ntiles), dim3(kTile), 0, s, mg, tiles, step, partial);
        if (nb_max == 5)
            hipLaunchKernelGGL((k_sor_mc<float, 5>), dim3(ntiles), dim3(kTile), 0, s, mg, tiles, step, partial);
    } else {
        hipLaunchKernelGGL((k_sor_mc<double, 3>), dim3(ntiles), dim3(kTile), 0, s, mg, tiles, step, partial);
        if (nb_max == 5)
            hipLaunchKernelGGL((k_sor_mc<double, 5>), dim3(ntiles), dim3(kTile), 0, s, mg, tiles, step, partial);
    }
    return hipGetLastError();
}

hipError_t launch_sor_finalize(const Inst1D *insts, int ninst, NewtonState *state, const double *partial,
                               double tol, hipStream_t s)
{
    hipLaunchKernelGGL(k_sor_finalize, dim3(ninst), dim3(64), 0, s, insts, ninst, state, partial, tol);
    return hipGetLastError();
}

hipError_t launch_sor_lex(const MGArgs &mg, int ninst, int nb_max, int zero_init, double tol, int prec,
                          hipStream_t s)
{
    const dim3 grid(ninst);   // one workgroup per instance
    if (prec == NMG_FP32_MG) {
        hipLaunchKernelGGL((k_sor_lex<float, 3>), grid, dim3(256), 0, s, mg, zero_init, tol);
        if (nb_max == 5) hipLaunchKernelGGL((k_sor_lex<float, 5>), grid, dim3(256), 0, s, mg, zero_init, tol);
    } else {
        hipLaunchKernelGGL((k_sor_lex<double, 3>), grid, dim3(256), 0, s, mg, zero_init, tol);
        if (nb_max == 5) hipLaunchKernelGGL((k_sor_lex<double, 5>), grid, dim3(256), 0, s, mg, zero_init, tol);
    }
    return hipGetLastError();
}

hipError_t launch_update1d(const MGArgs &mg, const Tile *tiles, int ntiles, int from_out, int prec, hipStream_t s)
{
    if (ntiles == 0) return hipSuccess;
    if (prec == NMG_FP32_MG)
        hipLaunchKernelGGL(k_update1d<float>, dim3(ntiles), dim3(kTile), 0, s, mg, tiles, from_out);
    else hipLaunchKernelGGL(k_update1d<double>, dim3(ntiles), dim3(kTile), 0, s, mg, tiles, from_out);
    return hipGetLastError();
}

hipError_t launch_interp_a2(const double *Uc, int nc, double *Uf, hipStream_t s)
{
    hipLaunchKernelGGL(k_interp_a2, dim3((nc + 255) / 256, 2), dim3(256), 0, s, Uc, nc, Uf);
    return hipGetLastError();
}

template <typename S, typename D>
__global__ void k_convert(const S *src, D *dst, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        dst[i] = (D)src[i];
}

// ---- launchers ---------------------------------------------------------------------------

hipError_t launch_coarsen1d(const MGArgs &mg, const Tile *tiles, int ntiles, int prec, hipStream_t s)
{
    if (ntiles == 0) return hipSuccess;
    if (prec == NMG_FP32_MG)
        hipLaunchKernelGGL(k_coarsen<float>, dim3(ntiles), dim3(kTile), 0, s, mg, tiles);
    else
        hipLaunchKernelGGL(k_coarsen<double>, dim3(ntiles), dim3(kTile), 0, s, mg, tiles);
    return hipGetLastError();
}

template <typename T>
static void launch_bottom_t(const MGArgs &mg, const int *inst_list, int n, int zero_init0, int final_update,
                            int nt, hipStream_t s)
{
    if (nt <= 256)
        hipLaunchKernelGGL((k_bottom<T, 256>), dim3(n), dim3(256), 0, s, mg, inst_list, zero_init0, final_update);
    else if (nt <= 512)
        hipLaunchKernelGGL((k_bottom<T, 512>), dim3(n), dim3(512), 0, s, mg, inst_list, zero_init0, final_update);
    else
        hipLaunchKernelGGL((k_bottom<T, 1024>), dim3(n), dim3(1024), 0, s, mg, inst_list, zero_init0, final_update);
}

hipError_t launch_bottom(const MGArgs &mg, const int *inst_list, int n, int zero_init0, int final_update,
                         int prec, int nt, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (nt != 256 && nt != 512 && nt != 1024) return hipErrorInvalidValue;
    if (prec == NMG_FP32_MG) launch_bottom_t<float>(mg, inst_list, n, zero_init0, final_update, nt, s);
    else launch_bottom_t<double>(mg, inst_list, n, zero_init0, final_update, nt, s);
    return hipGetLastError();
}

template <typename T, int NB, int TW>
static void launch_smooth_w(const MGArgs &mg, const Tile *tiles, int ntiles, int mode, int zero_init,
                            int final_update, int src_out, int reverse, hipStream_t s)
{
    if (mode == 0)
        hipLaunchKernelGGL((k_smooth<T, NB, 0, TW>), dim3(ntiles), dim3(TW), 0, s, mg, tiles, zero_init,
                           final_update, src_out, reverse);
    else if (mode == 1)
        hipLaunchKernelGGL((k_smooth<T, NB, 1, TW>), dim3(ntiles), dim3(TW), 0, s, mg, tiles, zero_init,
                           final_update, src_out, reverse);
    else
        hipLaunchKernelGGL((k_smooth<T, NB, 2, TW>), dim3(ntiles), dim3(TW), 0, s, mg, tiles, zero_init,
                           final_update, src_out, reverse);
}

template <typename T, int NB>
static void launch_smooth_t(const MGArgs &mg, const Tile *tiles, int ntiles, int mode, int zero_init,
                            int final_update, int src_out, int tile, int reverse, hipStream_t s)
{
    if (tile == kSmoothTileMax)
        launch_smooth_w<T, NB, kSmoothTileMax>(mg, tiles, ntiles, mode, zero_init, final_update, src_out, reverse, s);
    else
        launch_smooth_w<T, NB, kSmoothTile>(mg, tiles, ntiles, mode, zero_init, final_update, src_out, reverse, s);
}

hipError_t launch_smooth1d(const MGArgs &mg, const Tile *tiles, int ntiles, int nb_mask, int mode,
                           int zero_init, int final_update, int src_out, int prec, int tile, int reverse, hipStream_t s)
{
    if (ntiles == 0) return hipSuccess;
    if (tile != kSmoothTile && tile != kSmoothTileMax) return hipErrorInvalidValue;
    if (prec == NMG_FP32_MG) {
        if (nb_mask & 1) launch_smooth_t<float, 3>(mg, tiles, ntiles, mode, zero_init, final_update, src_out, tile, reverse, s);
        if (nb_mask & 2) launch_smooth_t<float, 5>(mg, tiles, ntiles, mode, zero_init, final_update, src_out, tile, reverse, s);
    } else {
        if (nb_mask & 1) launch_smooth_t<double, 3>(mg, tiles, ntiles, mode, zero_init, final_update, src_out, tile, reverse, s);
        if (nb_mask & 2) launch_smooth_t<double, 5>(mg, tiles, ntiles, mode, zero_init, final_update, src_out, tile, reverse, s);
    }
    return hipGetLastError();
}

hipError_t launch_convert(const void *src, int src_prec, void *dst, int dst_prec, long long n,
                          hipStream_t s)
{
    if (n == 0) return hipSuccess;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (src_prec == NMG_FP64 && dst_prec == NMG_FP64)
        hipLaunchKernelGGL((k_convert<double, double>), dim3(blocks), dim3(256), 0, s, (const double *)src, (double *)dst, n);
    else if (src_prec == NMG_FP64)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(blocks), dim3(256), 0, s, (const double *)src, (float *)dst, n);
    else if (dst_prec == NMG_FP64)
        hipLaunchKernelGGL((k_convert<float, double>), dim3(blocks), dim3(256), 0, s, (const float *)src, (double *)dst, n);
    else
        hipLaunchKernelGGL((k_convert<float, float>), dim3(blocks), dim3(256), 0, s, (const float *)src, (float *)dst, n);
    return hipGetLastError();
}

}  // namespace nmg
