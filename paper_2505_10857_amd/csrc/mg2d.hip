// Geometric multigrid for the 2D regularised Newton systems (section 4.2, eq. 22-25) on gfx950:
// coarse operators of eq. (24) (cross stencil -> five points on level 1, five points -> five
// points below), multicolour block SOR passes (eq. 22), restriction, injection prolongation,
// and Gaussian elimination with partial pivoting on the coarsest grid (dense, in LDS).
//
// Every level keeps its per-cell arrays in colour-blocked order (Perm2D): a colour pass of the
// smoother touches only the cells of one colour, and with the colours stored apart it reads them
// contiguously instead of pulling whole cache lines of interleaved colours.  One thread per cell
// or coarse cell; the sums run in the order of the definitions, so no result depends on the
// layout.
#include <algorithm>
#include <cstring>

#include "nmg_common.h"

namespace nmg {

template <typename T>
__device__ __forceinline__ double ld2(const T *p, long long i) { return (double)p[i]; }

// a load whose data will be evicted before it is read again (STREAM): the non-temporal hint
// keeps it out of the memory-side cache
template <bool STREAM, typename T>
__device__ __forceinline__ double lds2(const T *p)
{
    if (STREAM) return (double)__builtin_nontemporal_load(p);
    return (double)*p;
}

// stencil offsets: the cross of eq. (21) or the full 21 cells on the finest level, five points
// below (stencil_dx / stencil_dy)
__device__ __forceinline__ void stencil_off(int nb, int b, int &di, int &dj)
{
    di = stencil_dx(nb, b);
    dj = stencil_dy(nb, b);
}

__device__ __forceinline__ int find_off(int nb, int di, int dj)
{
    for (int b = 0; b < nb; b++) {
        int ox, oy;
        stencil_off(nb, b, ox, oy);
        if (ox == di && oy == dj) return b;
    }
    return -1;
}

__device__ __forceinline__ void inv3d(const double A[9], double B[9])
{
    const double c00 = A[4] * A[8] - A[5] * A[7];
    const double c01 = A[5] * A[6] - A[3] * A[8];
    const double c02 = A[3] * A[7] - A[4] * A[6];
    const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    B[0] = c00 / det;
    B[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    B[3] = c01 / det;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    B[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    B[6] = c02 / det;
    B[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / det;
}

// eq. (24), operator part, one thread per coarse cell: for each five-point offset, sum the fine
// blocks of the 2x2 children rows against the 2x2 children of the neighbour; then D^{-1}.
template <typename T>
__global__ void k_coarsen2d(T *mg, Level2D Lf, Level2D Lc)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int Jq = blockIdx.y;
    if (I >= Lc.nx || Jq >= Lc.ny) return;
    const long long nf = Lf.P.M, nc = Lc.P.M;
    const long long cc = perm2d(Lc.P, I, Jq);
    double D[9];
    for (int bc = 0; bc < 5; bc++) {
        int dP, dQ;
        stencil_off(5, bc, dP, dQ);
        const int P = I + dP, Q = Jq + dQ;
        double blk[9];
#pragma unroll
        for (int e = 0; e < 9; e++) blk[e] = 0.0;
        if (P >= 0 && P < Lc.nx && Q >= 0 && Q < Lc.ny) {
            for (int fj = 2 * Jq; fj <= 2 * Jq + 1; fj++)
                for (int fi = 2 * I; fi <= 2 * I + 1; fi++) {
                    const long long fc = perm2d(Lf.P, fi, fj);
                    for (int cj = 2 * Q; cj <= 2 * Q + 1; cj++)
                        for (int ci = 2 * P; ci <= 2 * P + 1; ci++) {
                            const int b = find_off(Lf.nb, ci - fi, cj - fj);
                            if (b < 0) continue;
#pragma unroll
                            for (int e = 0; e < 9; e++)
                                blk[e] = blk[e] + ld2(mg + Lf.J, (b * 9 + e) * nf + fc);
                        }
                }
        }
#pragma unroll
        for (int e = 0; e < 9; e++) {
            mg[Lc.J + (bc * 9 + e) * nc + cc] = (T)blk[e];
            if (bc == 0) D[e] = blk[e];
        }
    }
    double B[9];
    inv3d(D, B);
#pragma unroll
    for (int e = 0; e < 9; e++) mg[Lc.Dinv + e * nc + cc] = (T)B[e];
}

// `reps` consecutive passes of eq. (22) over the cells of one colour on one level with the
// NB-block stencil (C = 3 colours (i + j) mod 3 for the nine-block cross, 2 for five points, 9
// colours (i mod 3) + 3 (j mod 3) for the full 21 cells), thread p taking slot p of that colour's
// block (row p / W, k-th cell of the colour in the row).  Passes
// of one colour in a row see the same neighbour values, so the off-diagonal sum and D^{-1} r are
// formed once and the relaxation is applied `reps` times, each result rounded to the storage
// type as if it had been stored between the passes.  The stencil is unrolled so that every load
// of the cell's row is issued up front; neighbours outside the grid read the cell's own slot and
// are left out of the sum.
template <typename T, int NB, bool STREAM = false>
__device__ __forceinline__ void smooth_slot21(T *mg, const Level2D &L, int colour, double omega, int reps, long long p);

template <typename T, int NB, bool STREAM = false>
__device__ __forceinline__ void smooth_slot(T *mg, const Level2D &L, int colour, double omega, int reps, long long p)
{
    if constexpr (NB == 21) {
        smooth_slot21<T, NB, STREAM>(mg, L, colour, omega, reps, p);
        return;
    } else {
    constexpr int C = NB == 9 ? 3 : 2;
    const int W = L.P.W;
    const int j = (int)(p / W), k = (int)(p - (long long)j * W);
    const int i = ((colour - j) % C + C) % C + C * k;
    if (i >= L.nx) return;
    const long long n = L.P.M, cc = (long long)colour * L.P.ny * W + p;
    const T *Jr = mg + L.J + cc;
    const T *Ur = mg + L.dU;
    double x[NB][3];
    bool ok[NB];
#pragma unroll
    for (int b = 1; b < NB; b++) {
        int di, dj;
        stencil_off(NB, b, di, dj);
        const int pi = i + di, pj = j + dj;
        ok[b] = pi >= 0 && pi < L.nx && pj >= 0 && pj < L.ny;
        const int c2 = ((pi + pj) % C + C) % C;
        const int ic = ((c2 - pj) % C + C) % C;
        const long long q = ok[b] ? (long long)c2 * L.ny * W + (long long)pj * W + (pi - ic) / C : cc;
#pragma unroll
        for (int c = 0; c < 3; c++) x[b][c] = (double)Ur[c * n + q];
    }
    double a[NB][3];
#pragma unroll
    for (int b = 1; b < NB; b++)
#pragma unroll
        for (int c = 0; c < 3; c++)
            a[b][c] = lds2<STREAM>(Jr + (b * 9 + c * 3 + 0) * n) * x[b][0] + lds2<STREAM>(Jr + (b * 9 + c * 3 + 1) * n) * x[b][1] +
                      lds2<STREAM>(Jr + (b * 9 + c * 3 + 2) * n) * x[b][2];
    double r[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        r[c] = ld2(mg + L.rhs, c * n + cc);
#pragma unroll
        for (int b = 1; b < NB; b++)
            if (ok[b]) r[c] = r[c] + a[b][c];
    }
    double t[3];
#pragma unroll
    for (int c = 0; c < 3; c++)
        t[c] = lds2<STREAM>(mg + L.Dinv + (c * 3 + 0) * n + cc) * r[0] + lds2<STREAM>(mg + L.Dinv + (c * 3 + 1) * n + cc) * r[1] +
               lds2<STREAM>(mg + L.Dinv + (c * 3 + 2) * n + cc) * r[2];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        T d = mg[L.dU + c * n + cc];
        for (int q = 0; q < reps; q++) d = (T)((1.0 - omega) * (double)d - omega * t[c]);
        mg[L.dU + c * n + cc] = d;
    }
    }
}

// The same pass on the full 21-cell stencil with nine colours: thread p is cell
// (3 (p mod W) + colour mod 3, 3 (p / W) + colour / 3).  The off-diagonal sum runs block by block
// in stencil order (the order of eq. 22's sum as the oracle forms it), each block's three
// products added before the block joins the sum; the blocks' loads are independent of the sum,
// so they issue ahead of it.
template <typename T, int NB, bool STREAM>
__device__ __forceinline__ void smooth_slot21(T *mg, const Level2D &L, int colour, double omega, int reps, long long p)
{
    const int W = L.P.W;
    const int jr = (int)(p / W), k = (int)(p - (long long)jr * W);
    const int i = 3 * k + colour % 3, j = 3 * jr + colour / 3;
    if (i >= L.nx || j >= L.ny) return;
    const long long n = L.P.M, cc = (long long)colour * L.P.ny * W + p;
    const T *Jr = mg + L.J + cc;
    const T *Ur = mg + L.dU;
    double r[3];
#pragma unroll
    for (int c = 0; c < 3; c++) r[c] = ld2(mg + L.rhs, c * n + cc);
#pragma unroll
    for (int b = 1; b < 21; b++) {
        int di, dj;
        stencil_off(21, b, di, dj);
        const int pi = i + di, pj = j + dj;
        const bool ok = pi >= 0 && pi < L.nx && pj >= 0 && pj < L.ny;
        const long long q = ok ? perm2d(L.P, pi, pj) : cc;
        const double x0 = (double)Ur[q], x1 = (double)Ur[n + q], x2 = (double)Ur[2 * n + q];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const double a = lds2<STREAM>(Jr + (b * 9 + c * 3 + 0) * n) * x0 + lds2<STREAM>(Jr + (b * 9 + c * 3 + 1) * n) * x1 +
                             lds2<STREAM>(Jr + (b * 9 + c * 3 + 2) * n) * x2;
            if (ok) r[c] = r[c] + a;
        }
    }
    double t[3];
#pragma unroll
    for (int c = 0; c < 3; c++)
        t[c] = lds2<STREAM>(mg + L.Dinv + (c * 3 + 0) * n + cc) * r[0] + lds2<STREAM>(mg + L.Dinv + (c * 3 + 1) * n + cc) * r[1] +
               lds2<STREAM>(mg + L.Dinv + (c * 3 + 2) * n + cc) * r[2];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        T d = mg[L.dU + c * n + cc];
        for (int q = 0; q < reps; q++) d = (T)((1.0 - omega) * (double)d - omega * t[c]);
        mg[L.dU + c * n + cc] = d;
    }
}

template <typename T, int NB, bool STREAM>
__global__ void __launch_bounds__(256) k_smooth2d_pass(T *mg, Level2D L, int colour, double omega, int reps)
{
    const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (p >= (long long)L.P.ny * L.P.W) return;
    smooth_slot<T, NB, STREAM>(mg, L, colour, omega, reps, p);
}

// The same passes with each cell's three rows of eq. (22) on three lanes: wavefront c of a
// 192-thread workgroup forms row c (the off-diagonal sum in stencil order, as the per-cell form
// does) for 64 consecutive slots of the colour, so every wavefront reads one row of the blocks
// at consecutive addresses; the three sums meet in LDS, and lane c applies row c of D^{-1} and
// relaxes component c.  The same operations in the same order as smooth_slot, so the results
// are identical; three times the threads of the per-cell form, and a third of its loads per
// thread, keep more of a colour's cells in flight.
constexpr int kSplitCells = 64;

template <typename T, int NB, bool STREAM>
__global__ void __launch_bounds__(3 * kSplitCells) k_smooth2d_split(T *mg, Level2D L, int colour, double omega, int reps)
{
    __shared__ double sr[3][kSplitCells];
    constexpr int C = NB == 9 ? 3 : (NB == 21 ? 9 : 2);
    const int c = threadIdx.x / kSplitCells, lane = threadIdx.x % kSplitCells;
    const long long p = blockIdx.x * (long long)kSplitCells + lane;
    const int W = L.P.W;
    bool valid = p < (long long)L.P.ny * W;
    int i = 0, j = 0;
    if (valid) {
        const int jr = (int)(p / W), k = (int)(p - (long long)jr * W);
        if (C == 9) { i = 3 * k + colour % 3; j = 3 * jr + colour / 3; }
        else { j = jr; i = ((colour - j) % C + C) % C + C * k; }
        valid = i < L.nx && j < L.ny;
    }
    const long long n = L.P.M, cc = (long long)colour * L.P.ny * W + p;
    double r = 0.0;
    if (valid) {
        const T *Jr = mg + L.J + cc;
        const T *Ur = mg + L.dU;
        r = ld2(mg + L.rhs, c * n + cc);
#pragma unroll
        for (int b = 1; b < NB; b++) {
            int di, dj;
            stencil_off(NB, b, di, dj);
            const int pi = i + di, pj = j + dj;
            const bool ok = pi >= 0 && pi < L.nx && pj >= 0 && pj < L.ny;
            const long long q = ok ? perm2d(L.P, pi, pj) : cc;
            const double a = lds2<STREAM>(Jr + (b * 9 + c * 3 + 0) * n) * (double)Ur[q] +
                             lds2<STREAM>(Jr + (b * 9 + c * 3 + 1) * n) * (double)Ur[n + q] +
                             lds2<STREAM>(Jr + (b * 9 + c * 3 + 2) * n) * (double)Ur[2 * n + q];
            if (ok) r = r + a;
        }
    }
    sr[c][lane] = r;
    __syncthreads();
    if (!valid) return;
    const double t = lds2<STREAM>(mg + L.Dinv + (c * 3 + 0) * n + cc) * sr[0][lane] +
                     lds2<STREAM>(mg + L.Dinv + (c * 3 + 1) * n + cc) * sr[1][lane] +
                     lds2<STREAM>(mg + L.Dinv + (c * 3 + 2) * n + cc) * sr[2][lane];
    T d = mg[L.dU + c * n + cc];
    for (int q = 0; q < reps; q++) d = (T)((1.0 - omega) * (double)d - omega * t);
    mg[L.dU + c * n + cc] = d;
}

// ---- the four directional sweeps D1-D4 of section 4.2 (eq. 22 in a lexicographic order) ------

// eq. (22) for cell (i, j) in place, by a team of TEAM lanes (TEAM >= NB - 1, a power of two
// within one wavefront): lane m loads off-diagonal block b = m + 1 and the current dU of that
// neighbour and forms its product, all lanes at once (the loads of a hyperplane are one round
// trip, not NB - 1 of them); lane 0 of the team then adds the products to rhs in stencil order,
// skipping neighbours outside the grid, exactly the sequential sum, and writes
// dU <- (1 - omega) dU - omega D^{-1} r
template <typename T, int NB, int TEAM>
__device__ __forceinline__ void relax_cell_team(T *mg, const Level2D &L, int i, int j, double omega, int m)
{
    const long long n = L.P.M, cc = perm2d(L.P, i, j);
    const int b = m + 1;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if (b < NB) {
        int di, dj;
        stencil_off(NB, b, di, dj);
        const int pi = i + di, pj = j + dj;
        if (pi >= 0 && pi < L.nx && pj >= 0 && pj < L.ny) {
            const T *Jr = mg + L.J + cc;
            const T *Ur = mg + L.dU;
            const long long q = perm2d(L.P, pi, pj);
            const double x0 = (double)Ur[q], x1 = (double)Ur[n + q], x2 = (double)Ur[2 * n + q];
            a0 = (double)Jr[(b * 9 + 0) * n] * x0 + (double)Jr[(b * 9 + 1) * n] * x1 + (double)Jr[(b * 9 + 2) * n] * x2;
            a1 = (double)Jr[(b * 9 + 3) * n] * x0 + (double)Jr[(b * 9 + 4) * n] * x1 + (double)Jr[(b * 9 + 5) * n] * x2;
            a2 = (double)Jr[(b * 9 + 6) * n] * x0 + (double)Jr[(b * 9 + 7) * n] * x1 + (double)Jr[(b * 9 + 8) * n] * x2;
        }
    }
    double r0 = 0.0, r1 = 0.0, r2 = 0.0, Di[9], d0 = 0.0, d1 = 0.0, d2 = 0.0;
    if (m == 0) {
        r0 = ld2(mg + L.rhs, cc);
        r1 = ld2(mg + L.rhs, n + cc);
        r2 = ld2(mg + L.rhs, 2 * n + cc);
#pragma unroll
        for (int e = 0; e < 9; e++) Di[e] = ld2(mg + L.Dinv, e * n + cc);
        d0 = ld2(mg + L.dU, cc);
        d1 = ld2(mg + L.dU, n + cc);
        d2 = ld2(mg + L.dU, 2 * n + cc);
    }
#pragma unroll
    for (int bb = 1; bb < NB; bb++) {
        const double v0 = __shfl(a0, bb - 1, TEAM), v1 = __shfl(a1, bb - 1, TEAM), v2 = __shfl(a2, bb - 1, TEAM);
        int di, dj;
        stencil_off(NB, bb, di, dj);
        const int pi = i + di, pj = j + dj;
        if (pi >= 0 && pi < L.nx && pj >= 0 && pj < L.ny) {
            r0 = r0 + v0;
            r1 = r1 + v1;
            r2 = r2 + v2;
        }
    }
    if (m != 0) return;
    const double t0 = Di[0] * r0 + Di[1] * r1 + Di[2] * r2;
    const double t1 = Di[3] * r0 + Di[4] * r1 + Di[5] * r2;
    const double t2 = Di[6] * r0 + Di[7] * r1 + Di[8] * r2;
    mg[L.dU + cc] = (T)((1.0 - omega) * d0 - omega * t0);
    mg[L.dU + n + cc] = (T)((1.0 - omega) * d1 - omega * t1);
    mg[L.dU + 2 * n + cc] = (T)((1.0 - omega) * d2 - omega * t2);
}

// nu smoothing iterations of the sweeps D1 (x ascending, y ascending inside), D2 (x descending),
// D3 (both descending), D4 (y descending) on one level, by one workgroup.  In the coordinates
// (i', j') of a sweep (i' the outer index) a cell needs the new values of the coupled cells with
// A i' + j' smaller and the old ones of those with it larger (A = 1 for the cross and five-point
// stencils, 3 for the full 21 cells, whose couplings reach (1, -2)); the cells of one hyperplane
// A i' + j' = h are not coupled, so the hyperplanes run in order, each in parallel (a team of
// lanes per cell): the same result as the sequential sweep, bit for bit.
template <typename T, int NB>
__device__ void sweeps_level(T *mg, const Level2D &L, int nu, double omega)
{
    constexpr int A = NB == 21 ? 3 : 1;
    constexpr int TEAM = NB == 21 ? 32 : (NB == 9 ? 8 : 4);
    static_assert(TEAM >= NB - 1 && 64 % TEAM == 0, "a team per cell inside one wavefront");
    const int nx = L.nx, ny = L.ny, H = A * (nx - 1) + ny;
    const int team = (int)threadIdx.x / TEAM, m = (int)threadIdx.x % TEAM, teams = (int)blockDim.x / TEAM;
    for (int it = 0; it < nu; it++)
        for (int d = 0; d < 4; d++) {
            const bool fi = d == 1 || d == 2, fj = d >= 2;
            for (int h = 0; h < H; h++) {
                const int lo = h - (ny - 1) > 0 ? (h - (ny - 1) + A - 1) / A : 0;
                const int hi = nx - 1 < h / A ? nx - 1 : h / A;
                for (int k = lo + team; k <= hi; k += teams) {
                    const int jp = h - A * k;
                    relax_cell_team<T, NB, TEAM>(mg, L, fi ? nx - 1 - k : k, fj ? ny - 1 - jp : jp, omega, m);
                }
                __syncthreads();
            }
        }
}

template <typename T, int NB>
__global__ void __launch_bounds__(1024) k_sweeps2d(T *mg, Level2D L, int nu, double omega)
{
    sweeps_level<T, NB>(mg, L, nu, omega);
}

// eq. (24), right-hand side of coarse cell (I, Jq); also clears its dU.
// rhs + J dU of fine cell (fi, fj), the summand of eq. (24)'s restriction
template <typename T>
__device__ __forceinline__ void restrict_child(const T *mg, const Level2D &Lf, int fi, int fj, double a[3])
{
    const long long nf = Lf.P.M;
    const long long fc = perm2d(Lf.P, fi, fj);
#pragma unroll
    for (int c = 0; c < 3; c++) a[c] = ld2(mg + Lf.rhs, c * nf + fc);
    for (int b = 0; b < Lf.nb; b++) {
        int di, dj;
        stencil_off(Lf.nb, b, di, dj);
        const int pi = fi + di, pj = fj + dj;
        if (pi < 0 || pi >= Lf.nx || pj < 0 || pj >= Lf.ny) continue;
        const long long q = perm2d(Lf.P, pi, pj);
        const double x0 = ld2(mg + Lf.dU, q), x1 = ld2(mg + Lf.dU, nf + q), x2 = ld2(mg + Lf.dU, 2 * nf + q);
#pragma unroll
        for (int c = 0; c < 3; c++)
            a[c] = a[c] + (ld2(mg + Lf.J, (b * 9 + c * 3 + 0) * nf + fc) * x0 +
                           ld2(mg + Lf.J, (b * 9 + c * 3 + 1) * nf + fc) * x1 +
                           ld2(mg + Lf.J, (b * 9 + c * 3 + 2) * nf + fc) * x2);
    }
}

// coarse rhs = the four children's summands added in the order (2I, 2J), (2I+1, 2J), (2I, 2J+1),
// (2I+1, 2J+1); coarse dU = 0
template <typename T>
__device__ __forceinline__ void restrict_store(T *mg, const Level2D &Lc, int I, int Jq, const double a00[3],
                                               const double a10[3], const double a01[3], const double a11[3])
{
    const long long nc = Lc.P.M, cc = perm2d(Lc.P, I, Jq);
#pragma unroll
    for (int c = 0; c < 3; c++) {
        double sum = 0.0;
        sum = sum + a00[c];
        sum = sum + a10[c];
        sum = sum + a01[c];
        sum = sum + a11[c];
        mg[Lc.rhs + c * nc + cc] = (T)sum;
        mg[Lc.dU + c * nc + cc] = (T)0.0;
    }
}

template <typename T>
__device__ __forceinline__ void restrict_cell(T *mg, const Level2D &Lf, const Level2D &Lc, int I, int Jq)
{
    double a00[3], a10[3], a01[3], a11[3];
    restrict_child(mg, Lf, 2 * I, 2 * Jq, a00);
    restrict_child(mg, Lf, 2 * I + 1, 2 * Jq, a10);
    restrict_child(mg, Lf, 2 * I, 2 * Jq + 1, a01);
    restrict_child(mg, Lf, 2 * I + 1, 2 * Jq + 1, a11);
    restrict_store(mg, Lc, I, Jq, a00, a10, a01, a11);
}

// One workgroup per strip of two fine rows and kRX fine columns: a thread per fine cell forms its
// summand (consecutive lanes read consecutive slots of the colour-blocked arrays), then a thread
// per coarse cell adds its four children from LDS.
constexpr int kRX = 128;

template <typename T>
__global__ void __launch_bounds__(2 * kRX) k_restrict2d(T *mg, Level2D Lf, Level2D Lc)
{
    __shared__ double sa[3][2][kRX];
    const int t = threadIdx.x, r = t / kRX, x = t % kRX;
    const int fi = blockIdx.x * kRX + x, fj = 2 * blockIdx.y + r;
    if (fi < Lf.nx && fj < Lf.ny) {
        double a[3];
        restrict_child(mg, Lf, fi, fj, a);
#pragma unroll
        for (int c = 0; c < 3; c++) sa[c][r][x] = a[c];
    }
    __syncthreads();
    const int I = blockIdx.x * (kRX / 2) + t, Jq = blockIdx.y;
    if (t < kRX / 2 && I < Lc.nx && Jq < Lc.ny) {
        double a00[3], a10[3], a01[3], a11[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            a00[c] = sa[c][0][2 * t];
            a10[c] = sa[c][0][2 * t + 1];
            a01[c] = sa[c][1][2 * t];
            a11[c] = sa[c][1][2 * t + 1];
        }
        restrict_store(mg, Lc, I, Jq, a00, a10, a01, a11);
    }
}

// eq. (25): dU_fine += dU_coarse(parent)
template <typename T>
__device__ __forceinline__ void prolong_cell(T *mg, const Level2D &Lf, const Level2D &Lc, int i, int j)
{
    const long long nf = Lf.P.M, nc = Lc.P.M;
    const long long fc = perm2d(Lf.P, i, j), pc = perm2d(Lc.P, i >> 1, j >> 1);
#pragma unroll
    for (int c = 0; c < 3; c++)
        mg[Lf.dU + c * nf + fc] = (T)(ld2(mg + Lf.dU, c * nf + fc) + ld2(mg + Lc.dU, c * nc + pc));
}

template <typename T>
__global__ void k_prolong2d(T *mg, Level2D Lf, Level2D Lc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= Lf.nx || j >= Lf.ny) return;
    prolong_cell(mg, Lf, Lc, i, j);
}

// Coarsest level: Gaussian elimination with partial pivoting of the dense system sum J dU = -rhs
// (unknown (j*nx + i)*3 + c), split into a factorisation done once per operator and a solve per
// V-cycle.  The factorisation takes the pivots and eliminates exactly as the plain algorithm does
// (largest magnitude, first on ties; rows with a zero multiplier untouched) and keeps, in the
// workspace, the eliminated matrix with each multiplier in the place it eliminates (rows
// interchanged whole, multipliers included) and the row permutation.  The solve then applies the
// permutation to the right-hand side, the multipliers column by column (the same operations on
// the same values as eliminating the right-hand side alongside), and back substitution.
struct CoarseLU {
    double *A;    // [M][M]
    int *perm;    // [M]
};

__device__ __forceinline__ CoarseLU coarse_lu(double *base, int M) { return CoarseLU{base, (int *)(base + (long long)M * M)}; }

template <typename T>
__global__ void __launch_bounds__(256) k_coarse_factor2d(T *mg, Level2D L, double *lu_base)
{
    constexpr int MM = 3 * kMaxCoarse2D;
    __shared__ double A[MM * MM];
    __shared__ int perm[MM];
    __shared__ int piv_s;
    const int nx = L.nx, ny = L.ny, n = nx * ny, M = 3 * n;
    const long long Ms = L.P.M;
    const int t = threadIdx.x;
    for (int e = t; e < M * M; e += 256) A[e] = 0.0;
    for (int r = t; r < M; r += 256) perm[r] = r;
    __syncthreads();
    for (int e = t; e < n * L.nb; e += 256) {
        const int cell = e / L.nb, b = e % L.nb;
        const int i = cell % nx, j = cell / nx;
        int di, dj;
        stencil_off(L.nb, b, di, dj);
        const int pi = i + di, pj = j + dj;
        if (pi < 0 || pi >= nx || pj < 0 || pj >= ny) continue;
        const long long q = perm2d(L.P, i, j);
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++)
                A[(cell * 3 + r) * M + (pj * nx + pi) * 3 + c] = ld2(mg + L.J, (b * 9 + r * 3 + c) * Ms + q);
    }
    __syncthreads();
    for (int k = 0; k < M; k++) {
        if (t < 64) {            // pivot: largest |A[r][k]|, r >= k, the first one on ties
            int p = -1;
            double v = -1.0;
            for (int r = k + t; r < M; r += 64) {
                const double a = fabs(A[r * M + k]);
                if (a > v) { v = a; p = r; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double v2 = __shfl_xor(v, off, 64);
                const int p2 = __shfl_xor(p, off, 64);
                if (v2 > v || (v2 == v && p2 >= 0 && (p < 0 || p2 < p))) { v = v2; p = p2; }
            }
            if (t == 0) piv_s = p < 0 ? k : p;      // no comparable entry: keep the row
        }
        __syncthreads();
        const int p = piv_s;
        if (p != k) {
            for (int c = t; c < M; c += 256) {
                const double y = A[k * M + c];
                A[k * M + c] = A[p * M + c];
                A[p * M + c] = y;
            }
            if (t == 0) { const int y = perm[k]; perm[k] = perm[p]; perm[p] = y; }
        }
        __syncthreads();
        const double akk = A[k * M + k];
        // every thread reads column k before any row is updated
        double fr[(MM + 255) / 256];
#pragma unroll
        for (int q = 0; q < (MM + 255) / 256; q++) {
            const int r = k + 1 + t + 256 * q;
            fr[q] = r < M ? A[r * M + k] / akk : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < (MM + 255) / 256; q++) {
            const int r = k + 1 + t + 256 * q;
            if (r < M) A[r * M + k] = fr[q];
        }
        __syncthreads();
        const int w = M - k - 1;
        for (int e = t; e < w * w; e += 256) {
            const int r = k + 1 + e / w, c = k + 1 + e % w;
            const double f = A[r * M + k];
            if (f != 0.0) A[r * M + c] -= f * A[k * M + c];
        }
        __syncthreads();
    }
    const CoarseLU lu = coarse_lu(lu_base, M);
    for (int e = t; e < M * M; e += 256) lu.A[e] = A[e];
    for (int r = t; r < M; r += 256) lu.perm[r] = perm[r];
}

// solve with the factors of k_coarse_factor2d; A and x are LDS arrays of the calling workgroup
template <typename T>
__device__ __forceinline__ void coarse_apply(T *mg, const Level2D &L, const double *lu_base, double *A, double *x)
{
    const int nx = L.nx, n = nx * L.ny, M = 3 * n;
    const long long Ms = L.P.M;
    const int t = threadIdx.x, nt = blockDim.x;
    const CoarseLU lu = coarse_lu(const_cast<double *>(lu_base), M);
    for (int e = t; e < M * M; e += nt) A[e] = lu.A[e];
    for (int r = t; r < M; r += nt) {
        const int src = lu.perm[r], cell = src / 3;
        x[r] = -ld2(mg + L.rhs, (src % 3) * Ms + perm2d(L.P, cell % nx, cell / nx));
    }
    __syncthreads();
    for (int k = 0; k < M - 1; k++) {
        const double xk = x[k];
        for (int r = k + 1 + t; r < M; r += nt) {
            const double f = A[r * M + k];
            if (f != 0.0) x[r] -= f * xk;
        }
        __syncthreads();
    }
    // back substitution row by row, each row's sum over the later unknowns in ascending column
    // order (the order of a plain dense solve, so the result rounds like one); the rows depend on
    // each other in sequence, so one lane does it (at most 120 unknowns)
    if (t == 0) {
        for (int k = M - 1; k >= 0; k--) {
            double s = x[k];
            for (int c = k + 1; c < M; c++) s -= A[k * M + c] * x[c];
            x[k] = s / A[k * M + k];
        }
    }
    __syncthreads();
    for (int r = t; r < M; r += nt) {
        const int cell = r / 3;
        mg[L.dU + (r % 3) * Ms + perm2d(L.P, cell % nx, cell / nx)] = (T)x[r];
    }
}

// The bottom of a V-cycle in one workgroup: from level `first` (a small level) down to the
// coarsest and back, with every pass of Algorithm 2 on those levels (the same schedule of merged
// colour passes as the launches on the finer levels) separated by workgroup barriers instead of
// kernel boundaries.  Used for levels of at most kBottom2DCells cells, where a launch costs more
// than the pass itself.
struct Bottom2DArgs {
    Level2D L[kMaxLevels];
    int first, levels, nu1, nu2;
    double omega;
    const double *lu;
    int sweeps;          // smoother: 0 the multicolour schedule, 1 the directional sweeps D1-D4
};

// The merged colour passes of one five-point level of at most blockDim.x slots, with each
// thread's operator row (the four neighbour blocks, D^{-1} and the right-hand side) held in
// registers for all of them and dU in LDS (su, [3][M], each value rounded to the storage type as
// in memory): a pass then reads its neighbours from LDS instead of the level's arrays.  The
// operations of smooth_slot, in its order, so the results are the same bit for bit.
template <typename T>
__device__ void bottom_smooth5_resident(T *mg, const Level2D &L, int nu, double omega, double *su)
{
    constexpr int C = 2;
    const int W = L.P.W;
    const long long n = L.P.M, slots = (long long)L.P.ny * W;
    const int t = threadIdx.x;
    const int colour = (int)(t / slots);
    const long long p = t - colour * slots;
    const int j = (int)(p / W), k = (int)(p - (long long)j * W);
    const int i = ((colour - j) % C + C) % C + C * k;
    const bool mine = t < n && i < L.nx;
    const long long cc = t;   // colour * ny * W + p
    double Jb[5][9], Di[9], rh[3];
    int q[5];
    bool ok[5];
    if (mine) {
#pragma unroll
        for (int b = 1; b < 5; b++) {
            int di, dj;
            stencil_off(5, b, di, dj);
            const int pi = i + di, pj = j + dj;
            ok[b] = pi >= 0 && pi < L.nx && pj >= 0 && pj < L.ny;
            const int c2 = ((pi + pj) % C + C) % C;
            const int ic = ((c2 - pj) % C + C) % C;
            q[b] = ok[b] ? (int)((long long)c2 * L.ny * W + (long long)pj * W + (pi - ic) / C) : (int)cc;
#pragma unroll
            for (int e = 0; e < 9; e++) Jb[b][e] = ld2(mg + L.J, (b * 9 + e) * n + cc);
        }
#pragma unroll
        for (int e = 0; e < 9; e++) Di[e] = ld2(mg + L.Dinv, e * n + cc);
#pragma unroll
        for (int c = 0; c < 3; c++) rh[c] = ld2(mg + L.rhs, c * n + cc);
    }
    for (long long e = t; e < 3 * n; e += blockDim.x) su[e] = ld2(mg + L.dU, e);
    __syncthreads();
    int cur = -1, run = 0;
    for (int it = 0; it <= nu; it++) {
        for (int half = 0; half < 4; half++)
            for (int qq = 0; qq < C; qq++) {
                const bool last = it == nu;
                const int c = (half & 1) ? C - 1 - qq : qq;
                if (!last && c == cur) { run++; continue; }
                if (run > 0) {
                    if (mine && colour == cur) {
                        double x[5][3], a[5][3];
#pragma unroll
                        for (int b = 1; b < 5; b++)
#pragma unroll
                            for (int cm = 0; cm < 3; cm++) x[b][cm] = su[cm * n + q[b]];
#pragma unroll
                        for (int b = 1; b < 5; b++)
#pragma unroll
                            for (int cm = 0; cm < 3; cm++)
                                a[b][cm] = Jb[b][cm * 3 + 0] * x[b][0] + Jb[b][cm * 3 + 1] * x[b][1] + Jb[b][cm * 3 + 2] * x[b][2];
                        double r[3];
#pragma unroll
                        for (int cm = 0; cm < 3; cm++) {
                            r[cm] = rh[cm];
#pragma unroll
                            for (int b = 1; b < 5; b++)
                                if (ok[b]) r[cm] = r[cm] + a[b][cm];
                        }
#pragma unroll
                        for (int cm = 0; cm < 3; cm++) {
                            const double tt = Di[cm * 3 + 0] * r[0] + Di[cm * 3 + 1] * r[1] + Di[cm * 3 + 2] * r[2];
                            T d = (T)su[cm * n + cc];
                            for (int rr = 0; rr < run; rr++) d = (T)((1.0 - omega) * (double)d - omega * tt);
                            su[cm * n + cc] = (double)d;
                        }
                    }
                    __syncthreads();
                }
                if (last) {
                    for (long long e = t; e < 3 * n; e += blockDim.x) mg[L.dU + e] = (T)su[e];
                    __syncthreads();
                    return;
                }
                cur = c;
                run = 1;
            }
    }
}

// NBF: the stencil of the bottom's first level (the finest level when the whole hierarchy fits
// one workgroup, else a five-point level); the levels below it have five points.  Only the
// passes a launch can meet are compiled into it, which keeps the kernel's registers down.
// Five-point levels that fit the workgroup keep their operator in registers (su: LDS for dU),
// except in the kernel whose first level has the full 21-cell stencil, whose registers that
// would overflow.
template <typename T, int NBF>
__device__ void bottom_smooth(T *mg, const Level2D &L, int nu, double omega, int sweeps, double *su)
{
    if constexpr (NBF != 21) {
        if (!sweeps && L.nb == 5 && L.P.M <= (long long)blockDim.x) {
            bottom_smooth5_resident<T>(mg, L, nu, omega, su);
            return;
        }
    }
    if (sweeps) {
        if (NBF != 5 && L.nb == NBF) sweeps_level<T, NBF>(mg, L, nu, omega);
        else sweeps_level<T, 5>(mg, L, nu, omega);
        return;
    }
    const int C = L.P.C;
    const long long slots = (long long)L.P.ny * L.P.W;
    int cur = -1, run = 0;
    for (int it = 0; it <= nu; it++) {
        for (int half = 0; half < 4; half++)
            for (int q = 0; q < C; q++) {
                const bool last = it == nu;
                const int c = (half & 1) ? C - 1 - q : q;
                if (!last && c == cur) { run++; continue; }
                if (run > 0) {
                    for (long long p = threadIdx.x; p < slots; p += blockDim.x) {
                        if (NBF != 5 && L.nb == NBF) smooth_slot<T, NBF>(mg, L, cur, omega, run, p);
                        else smooth_slot<T, 5>(mg, L, cur, omega, run, p);
                    }
                    __syncthreads();
                }
                if (last) return;
                cur = c;
                run = 1;
            }
    }
}

template <typename T, int NBF>
__global__ void __launch_bounds__(512) k_bottom2d(T *mg, Bottom2DArgs B)
{
    constexpr int MM = 3 * kMaxCoarse2D;
    __shared__ double A[MM * MM];
    __shared__ double x[MM];
    __shared__ double su[3 * 512];   // dU of a five-point level held in LDS (at most 512 slots)
    const int last = B.levels - 1;
    for (int l = B.first; l < last; l++) {
        bottom_smooth<T, NBF>(mg, B.L[l], B.nu1, B.omega, B.sweeps, su);
        const Level2D &Lc = B.L[l + 1];
        for (int e = threadIdx.x; e < Lc.nx * Lc.ny; e += blockDim.x) restrict_cell(mg, B.L[l], Lc, e % Lc.nx, e / Lc.nx);
        __syncthreads();
    }
    coarse_apply(mg, B.L[last], B.lu, A, x);
    __syncthreads();
    for (int l = last - 1; l >= B.first; l--) {
        const Level2D &Lf = B.L[l];
        for (int e = threadIdx.x; e < Lf.nx * Lf.ny; e += blockDim.x) prolong_cell(mg, Lf, B.L[l + 1], e % Lf.nx, e / Lf.nx);
        __syncthreads();
        bottom_smooth<T, NBF>(mg, Lf, B.nu2, B.omega, B.sweeps, su);
    }
}

// inverse of the centre blocks of an FP64 level-0 operator in the natural order ([nb*9][n],
// block 0 first), written in the level's order
template <typename T>
__global__ void k_dinv2d(const double *J, T *Dinv, Level2D L0)
{
    const long long n = (long long)L0.nx * L0.ny;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
        double D[9], B[9];
#pragma unroll
        for (int e = 0; e < 9; e++) D[e] = J[e * n + c];
        inv3d(D, B);
        const long long q = perm2d(L0.P, (int)(c % L0.nx), (int)(c / L0.nx));
#pragma unroll
        for (int e = 0; e < 9; e++) Dinv[e * L0.P.M + q] = (T)B[e];
    }
}

// per-cell entries between the natural order [nent][n] and a level's order [nent][M]
template <typename S, typename D>
__global__ void k_permute2d(const S *src, D *dst, Level2D L, int nent, int to_level)
{
    const long long n = (long long)L.nx * L.ny, total = n * nent;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        const long long c = e % n, a = e / n;
        const long long q = perm2d(L.P, (int)(c % L.nx), (int)(c / L.nx));
        if (to_level) dst[a * L.P.M + q] = (D)src[e];
        else dst[e] = (D)src[a * L.P.M + q];
    }
}

template <typename T>
__global__ void k_fill(T *p, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = (T)0.0;
}

// eq. (14): U <- U + tau dU (skipped once the Newton iteration has stopped); U in the natural
// order [3][ny][nx]
template <typename T>
__global__ void k_update2d(double *U, const T *mg, Level2D L0, double tau, const NewtonState *S)
{
    if (S && !S->active) return;
    const long long n = (long long)L0.nx * L0.ny;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < 3 * n; e += (long long)gridDim.x * blockDim.x) {
        const long long c = e % n, comp = e / n;
        const long long q = perm2d(L0.P, (int)(c % L0.nx), (int)(c / L0.nx));
        U[e] = U[e] + tau * ld2(mg + L0.dU, comp * L0.P.M + q);
    }
}

// res from the tile partials, Newton counter and stopping test (Algorithm 1)
__global__ void __launch_bounds__(256) k_state2d(const double *partial, int ntiles, long long ncells, double tol,
                                                 int n_max, NewtonState *S, double *hist, int max_hist, int init)
{
    __shared__ double red[4];
    double v = 0.0;
    for (int k = threadIdx.x; k < ntiles; k += 256) v += partial[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double res = (red[0] + red[1] + red[2] + red[3]) / (double)ncells;
    if (init) {
        S->res = res; S->n = 0; S->active = 1; S->status = NMG_NOT_CONVERGED;
        if (!(res == res) || res > 1e300) { S->active = 0; S->status = NMG_ENONFINITE; }
        return;
    }
    if (!S->active) return;
    S->res = res;
    if (hist && S->n < max_hist) hist[S->n] = res;
    S->n += 1;
    if (!(res == res) || res > 1e300) { S->active = 0; S->status = NMG_ENONFINITE; }
    else if (res < tol) { S->active = 0; S->status = NMG_OK; }
    else if (S->n >= n_max) { S->active = 0; S->status = NMG_NOT_CONVERGED; }
}

// ---- nested iteration: Appendix A in two dimensions (eq. A.3) ------------------------------

// Eq. (A.2) from three consecutive coarse values um, u0, up of a line centred at cell k, for
// half h (0 or 1) of coarse cell j: in the interior j = k and the half's average of the quadratic
// (A.1) has the weights (1/8, 1, -1/8) or (-1/8, 1, 1/8); the first and last cell of the line
// (j = 0, k = 1 or j = n-1, k = n-2) average the quadratic centred one cell inward over their
// half.
__device__ __forceinline__ double a2_from3(double um, double u0, double up, int j, int k, int h)
{
    if (j == k) {
        if (h == 0) return um / 8.0 + u0 - up / 8.0;
        return -um / 8.0 + u0 + up / 8.0;
    }
    const double a = (up - um) / 2.0;
    const double b = (um - 2.0 * u0 + up) / 2.0;
    const double lo = (double)(j - k) - 0.5 + 0.5 * h, hi = lo + 0.5;
    const double m1 = (lo + hi) / 2.0;                      // mean of xi over the half
    const double m2 = (lo * lo + lo * hi + hi * hi) / 3.0;  // mean of xi^2
    return u0 + a * m1 + b * (m2 - 1.0 / 12.0);
}

__device__ __forceinline__ int a2_centre(int j, int n) { return j >= 1 && j <= n - 2 ? j : (j == 0 ? 1 : n - 2); }

// Fine cell (fi, fj) of component c: the polynomial of eq. (A.3) is the tensor product of the
// quadratics (A.1), so its average over a quarter of a coarse cell is eq. (A.2) along x in the
// three coarse rows it needs, then eq. (A.2) along y of those three values (the same operations
// in the same order as refining every coarse row in x first and every fine column in y after).
__global__ void __launch_bounds__(256) k_interp_a3(const double *Uc, int nxc, int nyc, double *Uf)
{
    const int fi = blockIdx.x * blockDim.x + threadIdx.x, fj = blockIdx.y, c = blockIdx.z;
    const int nxf = 2 * nxc;
    if (fi >= nxf) return;
    const double *u = Uc + (long long)c * nyc * nxc;
    const int ic = fi >> 1, hx = fi & 1, jc = fj >> 1, hy = fj & 1;
    const int kx = a2_centre(ic, nxc), ky = a2_centre(jc, nyc);
    double t[3];
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const double *row = u + (long long)(ky - 1 + q) * nxc;
        t[q] = a2_from3(row[kx - 1], row[kx], row[kx + 1], ic, kx, hx);
    }
    Uf[((long long)c * 2 * nyc + fj) * nxf + fi] = a2_from3(t[0], t[1], t[2], jc, ky, hy);
}

hipError_t launch_interp_a3(const double *Uc, int nxc, int nyc, double *Uf, hipStream_t s)
{
    if (nxc < 3 || nyc < 3 || 2 * (long long)nyc > 65535) return hipErrorInvalidValue;   // grid.y holds the fine rows
    dim3 grid((2 * nxc + 255) / 256, 2 * nyc, 3);
    hipLaunchKernelGGL(k_interp_a3, grid, dim3(256), 0, s, Uc, nxc, nyc, Uf);
    return hipGetLastError();
}

// ---- launchers ---------------------------------------------------------------------------

#define DISPATCH(prec, KER, grid, block, ...)                                                      \
    do {                                                                                           \
        if ((prec) == NMG_FP32_MG) hipLaunchKernelGGL(KER<float>, grid, block, 0, s, (float *)mg, __VA_ARGS__); \
        else hipLaunchKernelGGL(KER<double>, grid, block, 0, s, (double *)mg, __VA_ARGS__);       \
    } while (0)

hipError_t launch_coarsen2d(void *mg, const Level2D &Lf, const Level2D &Lc, int prec, hipStream_t s)
{
    dim3 grid((Lc.nx + 63) / 64, Lc.ny);
    DISPATCH(prec, k_coarsen2d, grid, dim3(64), Lf, Lc);
    return hipGetLastError();
}

// The full stencil's passes take the three-lanes-per-cell form: a colour holds a ninth of the
// cells, too few for one thread per cell to fill the chip, and a cell's 20 off-diagonal blocks
// are a long chain of loads for one thread (measured on the 1024 x 512 wedge: 35 against 56 ms
// per FP64 V-cycle, 30 against 62 ms in FP32).  The cross and five-point passes keep one thread
// per cell, whose loads all issue up front (13.2 against 13.7 ms FP64, 8.3 against 10.8 ms FP32
// per J9 V-cycle).  Both forms give identical results; alt (a schedule choice) swaps them.
template <typename T, int NB, bool STREAM>
static void smooth2d_launch(T *mg, const Level2D &L, int colour, int reps, double omega, hipStream_t s, bool alt)
{
    const long long slots = (long long)L.P.ny * L.P.W;
    if ((NB == 21) != alt) {
        dim3 grid((unsigned)((slots + kSplitCells - 1) / kSplitCells));
        hipLaunchKernelGGL((k_smooth2d_split<T, NB, STREAM>), grid, dim3(3 * kSplitCells), 0, s, mg, L, colour, omega, reps);
    } else {
        dim3 grid((unsigned)((slots + 255) / 256));
        hipLaunchKernelGGL((k_smooth2d_pass<T, NB, STREAM>), grid, dim3(256), 0, s, mg, L, colour, omega, reps);
    }
}

hipError_t launch_smooth2d_pass(void *mg, const Level2D &L, int colour, int reps, double omega, int prec,
                               hipStream_t s, int sched)
{
    if (L.P.C != (L.nb == 9 ? 3 : (L.nb == 21 ? 9 : 2))) return hipErrorInvalidValue;
    const bool f32 = prec == NMG_FP32_MG;
    const size_t vsz = f32 ? 4 : 8;
    const bool alt = (sched & (L.nb == 5 ? NMG_SCHED2D_ALT_COARSE : NMG_SCHED2D_ALT_FINEST)) != 0;
    const bool big = !(sched & NMG_SCHED2D_NO_STREAM) && (size_t)L.nb * 9 * (size_t)L.P.M * vsz > kMemCacheBytes;
    // Operators larger than the memory-side cache: on the cross stencil the symmetric schedule
    // returns to colour 1 every other run and to colours 0 and 2 every fourth, so colours 0 and 2
    // stream their rows and leave the cache to colour 1's; with nine colours a colour's rows come
    // back only after the eight others have streamed theirs, so every pass streams.
    const bool stream = big && (L.nb == 21 || (L.nb == 9 && colour != 1));
    if (L.nb == 21) {
        if (f32) { if (stream) smooth2d_launch<float, 21, true>((float *)mg, L, colour, reps, omega, s, alt);
                   else smooth2d_launch<float, 21, false>((float *)mg, L, colour, reps, omega, s, alt); }
        else { if (stream) smooth2d_launch<double, 21, true>((double *)mg, L, colour, reps, omega, s, alt);
               else smooth2d_launch<double, 21, false>((double *)mg, L, colour, reps, omega, s, alt); }
    } else if (L.nb == 9) {
        if (f32) { if (stream) smooth2d_launch<float, 9, true>((float *)mg, L, colour, reps, omega, s, alt);
                   else smooth2d_launch<float, 9, false>((float *)mg, L, colour, reps, omega, s, alt); }
        else { if (stream) smooth2d_launch<double, 9, true>((double *)mg, L, colour, reps, omega, s, alt);
               else smooth2d_launch<double, 9, false>((double *)mg, L, colour, reps, omega, s, alt); }
    } else {
        if (f32) smooth2d_launch<float, 5, false>((float *)mg, L, colour, reps, omega, s, alt);
        else smooth2d_launch<double, 5, false>((double *)mg, L, colour, reps, omega, s, alt);
    }
    return hipGetLastError();
}

hipError_t launch_restrict2d(void *mg, const Level2D &Lf, const Level2D &Lc, int prec, hipStream_t s)
{
    dim3 grid((Lf.nx + kRX - 1) / kRX, Lc.ny);
    DISPATCH(prec, k_restrict2d, grid, dim3(2 * kRX), Lf, Lc);
    return hipGetLastError();
}

hipError_t launch_prolong2d(void *mg, const Level2D &Lf, const Level2D &Lc, int prec, hipStream_t s)
{
    dim3 grid((Lf.nx + 63) / 64, (Lf.ny + 3) / 4);
    DISPATCH(prec, k_prolong2d, grid, dim3(64, 4), Lf, Lc);
    return hipGetLastError();
}

hipError_t launch_coarse_factor2d(void *mg, const Level2D &L, double *lu, int prec, hipStream_t s)
{
    DISPATCH(prec, k_coarse_factor2d, dim3(1), dim3(256), L, lu);
    return hipGetLastError();
}

hipError_t launch_sweeps2d(void *mg, const Level2D &L, int nu, double omega, int prec, hipStream_t s)
{
    const bool f32 = prec == NMG_FP32_MG;
    if (L.nb == 21) {
        if (f32) hipLaunchKernelGGL((k_sweeps2d<float, 21>), dim3(1), dim3(1024), 0, s, (float *)mg, L, nu, omega);
        else hipLaunchKernelGGL((k_sweeps2d<double, 21>), dim3(1), dim3(1024), 0, s, (double *)mg, L, nu, omega);
    } else if (L.nb == 9) {
        if (f32) hipLaunchKernelGGL((k_sweeps2d<float, 9>), dim3(1), dim3(1024), 0, s, (float *)mg, L, nu, omega);
        else hipLaunchKernelGGL((k_sweeps2d<double, 9>), dim3(1), dim3(1024), 0, s, (double *)mg, L, nu, omega);
    } else {
        if (f32) hipLaunchKernelGGL((k_sweeps2d<float, 5>), dim3(1), dim3(1024), 0, s, (float *)mg, L, nu, omega);
        else hipLaunchKernelGGL((k_sweeps2d<double, 5>), dim3(1), dim3(1024), 0, s, (double *)mg, L, nu, omega);
    }
    return hipGetLastError();
}

hipError_t launch_bottom2d(void *mg, const Level2D *levels, int first, int nlev, int nu1, int nu2, double omega,
                           const double *lu, int prec, hipStream_t s, int sweeps)
{
    if (first < 0 || first >= nlev || nlev > kMaxLevels) return hipErrorInvalidValue;
    Bottom2DArgs B;
    memset(&B, 0, sizeof(B));
    for (int l = 0; l < nlev; l++) B.L[l] = levels[l];
    B.first = first;
    B.levels = nlev;
    B.nu1 = nu1;
    B.nu2 = nu2;
    B.omega = omega;
    B.lu = lu;
    B.sweeps = sweeps;
    const int nbf = levels[first].nb;
    const bool f32 = prec == NMG_FP32_MG;
    float *mf = (float *)mg;
    double *md = (double *)mg;
    if (nbf == 21) {
        if (f32) hipLaunchKernelGGL((k_bottom2d<float, 21>), dim3(1), dim3(512), 0, s, mf, B);
        else hipLaunchKernelGGL((k_bottom2d<double, 21>), dim3(1), dim3(512), 0, s, md, B);
    } else if (nbf == 9) {
        if (f32) hipLaunchKernelGGL((k_bottom2d<float, 9>), dim3(1), dim3(512), 0, s, mf, B);
        else hipLaunchKernelGGL((k_bottom2d<double, 9>), dim3(1), dim3(512), 0, s, md, B);
    } else {
        if (f32) hipLaunchKernelGGL((k_bottom2d<float, 5>), dim3(1), dim3(512), 0, s, mf, B);
        else hipLaunchKernelGGL((k_bottom2d<double, 5>), dim3(1), dim3(512), 0, s, md, B);
    }
    return hipGetLastError();
}

hipError_t launch_fill(void *p, int prec, long long n, hipStream_t s)
{
    int blocks = (int)std::min<long long>((n + 255) / 256, 4096);
    if (blocks < 1) return hipSuccess;
    if (prec == NMG_FP32_MG) hipLaunchKernelGGL(k_fill<float>, dim3(blocks), dim3(256), 0, s, (float *)p, n);
    else hipLaunchKernelGGL(k_fill<double>, dim3(blocks), dim3(256), 0, s, (double *)p, n);
    return hipGetLastError();
}

hipError_t launch_update2d(double *U, const void *mg, const Level2D &L0, double tau, const NewtonState *state,
                           int prec, hipStream_t s)
{
    const long long n = 3LL * L0.nx * L0.ny;
    int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    if (prec == NMG_FP32_MG)
        hipLaunchKernelGGL(k_update2d<float>, dim3(blocks), dim3(256), 0, s, U, (const float *)mg, L0, tau, state);
    else
        hipLaunchKernelGGL(k_update2d<double>, dim3(blocks), dim3(256), 0, s, U, (const double *)mg, L0, tau, state);
    return hipGetLastError();
}

hipError_t launch_dinv2d(const double *J, void *Dinv, const Level2D &L0, int prec, hipStream_t s)
{
    const long long n = (long long)L0.nx * L0.ny;
    int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    if (prec == NMG_FP32_MG) hipLaunchKernelGGL(k_dinv2d<float>, dim3(blocks), dim3(256), 0, s, J, (float *)Dinv, L0);
    else hipLaunchKernelGGL(k_dinv2d<double>, dim3(blocks), dim3(256), 0, s, J, (double *)Dinv, L0);
    return hipGetLastError();
}

hipError_t launch_permute2d(const void *src, int src_prec, void *dst, int dst_prec, const Level2D &L, int nent,
                            int to_level, hipStream_t s)
{
    const long long total = (long long)L.nx * L.ny * nent;
    int blocks = (int)std::min<long long>((total + 255) / 256, 16384);
    if (blocks < 1) return hipSuccess;
    const bool s32 = src_prec == NMG_FP32_MG, d32 = dst_prec == NMG_FP32_MG;
    if (!s32 && !d32)
        hipLaunchKernelGGL((k_permute2d<double, double>), dim3(blocks), dim3(256), 0, s, (const double *)src,
                           (double *)dst, L, nent, to_level);
    else if (!s32)
        hipLaunchKernelGGL((k_permute2d<double, float>), dim3(blocks), dim3(256), 0, s, (const double *)src,
                           (float *)dst, L, nent, to_level);
    else if (!d32)
        hipLaunchKernelGGL((k_permute2d<float, double>), dim3(blocks), dim3(256), 0, s, (const float *)src,
                           (double *)dst, L, nent, to_level);
    else
        hipLaunchKernelGGL((k_permute2d<float, float>), dim3(blocks), dim3(256), 0, s, (const float *)src,
                           (float *)dst, L, nent, to_level);
    return hipGetLastError();
}

hipError_t launch_state2d(const double *partial, int ntiles, long long ncells, double tol, int n_max,
                          NewtonState *state, double *hist, int max_hist, int init, hipStream_t s)
{
    hipLaunchKernelGGL(k_state2d, dim3(1), dim3(256), 0, s, partial, ntiles, ncells, tol, n_max, state, hist,
                       max_hist, init);
    return hipGetLastError();
}

}  // namespace nmg
