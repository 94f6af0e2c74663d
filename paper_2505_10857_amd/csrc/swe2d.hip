// 2D finite-volume residual (section 4.1, eq. 20) with characteristic WENO3, Gauss quadrature
// along faces and the tensor Gauss source, and its finite-difference Jacobian on the cross
// stencil of eq. (21), for gfx950.
//
// A 32x8 tile of cells stages U for its cells plus two halo cells on every side in LDS; every
// thread evaluates its cell's residual from LDS.  Ghost cells are not stored: a stencil access
// outside the grid maps to the interior cell it is built from (copy, mirror) and applies the
// boundary rule, so the finite-difference Jacobian perturbs ghosts together with the interior
// cell they follow.  The arithmetic is that of the formulas in their printed order, without FMA
// contraction, and correctly rounded division and square root, so the residual is reproducible
// bit for bit; with the 1e-6 perturbation of the 2D Jacobian anything less would be amplified
// a million times.
#include "nmg_common.h"

namespace nmg {

constexpr int kTX = 32, kTY = 8;                       // tile of cells
constexpr int kSX = kTX + 4, kSY = kTY + 4;            // staged region (halo 2)

struct Pert {                  // a perturbation of component m of cell (pi, pj) by eps
    int pi, pj, m;
    double eps;
};

__device__ __forceinline__ double weno_p2(double um, double u0, double up)
{
    double c0 = 1.5 * u0 - 0.5 * up;
    double c1 = 0.5 * um + 0.5 * u0;
    double b0 = (up - u0) * (up - u0);
    double b1 = (u0 - um) * (u0 - um);
    double a0 = (1.0 / 3.0) / ((kZeta + b0) * (kZeta + b0));
    double a1 = (2.0 / 3.0) / ((kZeta + b1) * (kZeta + b1));
    double w0 = a0 / (a0 + a1);
    double w1 = a1 / (a0 + a1);
    return w0 * c0 + w1 * c1;
}

__device__ __forceinline__ double weno_m2(double um, double u0, double up)
{
    double c0 = 0.5 * u0 + 0.5 * up;
    double c1 = -0.5 * um + 1.5 * u0;
    double b0 = (up - u0) * (up - u0);
    double b1 = (u0 - um) * (u0 - um);
    double a0 = (2.0 / 3.0) / ((kZeta + b0) * (kZeta + b0));
    double a1 = (1.0 / 3.0) / ((kZeta + b1) * (kZeta + b1));
    double w0 = a0 / (a0 + a1);
    double w1 = a1 / (a0 + a1);
    return w0 * c0 + w1 * c1;
}

// Staged state of one tile: s[c][y][x] for cells (i0-2+x, j0-2+y).
struct Stage {
    const double *s;
    int i0, j0;
};

__device__ __forceinline__ double stage_at(const Stage &S, int c, int i, int j)
{
    return S.s[(c * kSY + (j - S.j0 + 2)) * kSX + (i - S.i0 + 2)];
}

// Cell (i, j) of the (perturbed) state, ghosts included: y sides first, then x sides.
__device__ __forceinline__ void cell2(const Inst2D &I, const Stage &S, const Pert &P, int i, int j,
                                      double out[3])
{
    int ii = i, jj = j, flip_u = 0, flip_v = 0, state = -1, set_h = -1, set_q = -1;
    if (j < 0 || j >= I.Ny) {
        const int side = j < 0 ? 2 : 3;
        int kind = I.bc_kind[side];
        if (side == 2 && I.bc_kind[2] == NMG_BC_WALL && I.wall_x > I.x0) {
            double xc = I.x0 + (i + 0.5) * I.dx;
            kind = xc < I.wall_x ? NMG_BC_EXTRAP : NMG_BC_WALL;
        }
        const int b = j < 0 ? 0 : I.Ny - 1;
        const int m = j < 0 ? -1 - j : 2 * I.Ny - 1 - j;
        jj = b;
        if (kind == NMG_BC_WALL) { jj = m; flip_v = 1; }
        else if (kind == NMG_BC_STATE) state = side;
        else if (kind == NMG_BC_DISCHARGE) set_q = side;
        else if (kind == NMG_BC_DEPTH) set_h = side;
    }
    if (i < 0 || i >= I.Nx) {
        const int side = i < 0 ? 0 : 1;
        const int kind = I.bc_kind[side];
        const int b = i < 0 ? 0 : I.Nx - 1;
        const int m = i < 0 ? -1 - i : 2 * I.Nx - 1 - i;
        ii = b;
        if (kind == NMG_BC_WALL) { ii = m; flip_u = 1; }
        else if (kind == NMG_BC_STATE) state = side;
        else if (kind == NMG_BC_DISCHARGE) set_q = side;
        else if (kind == NMG_BC_DEPTH) set_h = side;
    }
    if (state >= 0) {
        out[0] = I.bc_h[state];
        out[1] = I.bc_h[state] * I.bc_u[state];
        out[2] = I.bc_h[state] * I.bc_v[state];
        return;
    }
    const bool hit = ii == P.pi && jj == P.pj;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const double x = stage_at(S, c, ii, jj);
        out[c] = (hit && c == P.m) ? x + P.eps : x;
    }
    if (flip_u) out[1] = -out[1];
    if (flip_v) out[2] = -out[2];
    if (set_h >= 0) out[0] = I.bc_h[set_h];
    if (set_q >= 0) {
        if (set_q < 2) out[1] = I.bc_q[set_q];
        else out[2] = I.bc_q[set_q];
    }
}

// Characteristic WENO3 state at the face between cells a and a+1 of line k (dir 0: row k; dir 1:
// column k), from cell a (which = 0) or a+1 (which = 1); the basis is the eigensystem of the
// face-normal flux Jacobian at the mean of the two cells.
__device__ void face_state2(const Inst2D &I, const Stage &S, const Pert &P, int dir, int k, int a,
                            int which, double out[3])
{
    double Ua[3], Ub[3], Us[3];
    if (dir == 0) { cell2(I, S, P, a, k, Ua); cell2(I, S, P, a + 1, k, Ub); }
    else { cell2(I, S, P, k, a, Ua); cell2(I, S, P, k, a + 1, Ub); }
#pragma unroll
    for (int c = 0; c < 3; c++) Us[c] = 0.5 * (Ua[c] + Ub[c]);
    const double h = Us[0];
    const double u = Us[1] / h;
    const double v = Us[2] / h;
    const double cc = sqrt(I.g * h);
    const double un = dir == 0 ? u : v;
    const double i2c = 1.0 / (2.0 * cc);
    double L[3][3], R[3][3];
    if (dir == 0) {
        L[0][0] = (un + cc) * i2c; L[0][1] = -i2c; L[0][2] = 0.0;
        L[1][0] = -v;              L[1][1] = 0.0;  L[1][2] = 1.0;
        L[2][0] = -(un - cc) * i2c; L[2][1] = i2c; L[2][2] = 0.0;
        R[0][0] = 1.0;     R[0][1] = 0.0; R[0][2] = 1.0;
        R[1][0] = un - cc; R[1][1] = 0.0; R[1][2] = un + cc;
        R[2][0] = v;       R[2][1] = 1.0; R[2][2] = v;
    } else {
        L[0][0] = (un + cc) * i2c; L[0][1] = 0.0; L[0][2] = -i2c;
        L[1][0] = -u;              L[1][1] = 1.0; L[1][2] = 0.0;
        L[2][0] = -(un - cc) * i2c; L[2][1] = 0.0; L[2][2] = i2c;
        R[0][0] = 1.0;     R[0][1] = 0.0; R[0][2] = 1.0;
        R[1][0] = u;       R[1][1] = 1.0; R[1][2] = u;
        R[2][0] = un - cc; R[2][1] = 0.0; R[2][2] = un + cc;
    }
    const int m = which ? a + 1 : a;
    double St[3][3];
#pragma unroll
    for (int s = 0; s < 3; s++) {
        if (dir == 0) cell2(I, S, P, m - 1 + s, k, St[s]);
        else cell2(I, S, P, k, m - 1 + s, St[s]);
    }
    double W[3][3], w[3];
#pragma unroll
    for (int s = 0; s < 3; s++)
#pragma unroll
        for (int f = 0; f < 3; f++)
            W[s][f] = L[f][0] * St[s][0] + L[f][1] * St[s][1] + L[f][2] * St[s][2];
#pragma unroll
    for (int f = 0; f < 3; f++)
        w[f] = which ? weno_p2(W[0][f], W[1][f], W[2][f]) : weno_m2(W[0][f], W[1][f], W[2][f]);
#pragma unroll
    for (int c = 0; c < 3; c++) out[c] = R[c][0] * w[0] + R[c][1] * w[1] + R[c][2] * w[2];
}

__device__ __forceinline__ void flux2(const double U[3], int dir, double g, double F[3])
{
    const double h = U[0];
    const double u = U[1] / h;
    const double v = U[2] / h;
    if (dir == 0) {
        F[0] = U[1];
        F[1] = U[1] * u + 0.5 * g * h * h;
        F[2] = U[1] * v;
    } else {
        F[0] = U[2];
        F[1] = U[2] * u;
        F[2] = U[2] * v + 0.5 * g * h * h;
    }
}

__device__ __forceinline__ void llf2(const double UL[3], const double UR[3], int dir, double g, double F[3])
{
    double FL[3], FR[3];
    flux2(UL, dir, g, FL);
    flux2(UR, dir, g, FR);
    const double unL = UL[1 + dir] / UL[0], unR = UR[1 + dir] / UR[0];
    const double sL = fabs(unL) + sqrt(g * UL[0]);
    const double sR = fabs(unR) + sqrt(g * UR[0]);
    const double a = sL > sR ? sL : sR;
#pragma unroll
    for (int c = 0; c < 3; c++) F[c] = 0.5 * (FL[c] + FR[c] - a * (UR[c] - UL[c]));
}

// The quadratic through three face averages at the two Gauss points (its curvature term is zero
// there): P = V0 + t (Vp - Vm) / 2, t = -+1/(2 sqrt 3).
__device__ __forceinline__ void gauss_line2(const double Vm[3], const double V0[3], const double Vp[3],
                                            double P[2][3])
{
    const double t0 = -1.0 / (2.0 * sqrt(3.0)), t1 = 1.0 / (2.0 * sqrt(3.0));
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const double slope = (Vp[c] - Vm[c]) * 0.5;
        P[0][c] = V0[c] + t0 * slope;
        P[1][c] = V0[c] + t1 * slope;
    }
}

// Edge-averaged LLF flux through a face (two-point Gauss rule along it); also the depths of the
// minus and plus states at the two Gauss points.
__device__ void face_flux2(const Inst2D &I, const Stage &S, const Pert &P, int dir, int line, int a,
                           double F[3], double hm[2], double hp[2])
{
    double Vm[3][3], Vp[3][3], Pm[2][3], Pp[2][3];
#pragma unroll
    for (int s = 0; s < 3; s++) {
        face_state2(I, S, P, dir, line - 1 + s, a, 0, Vm[s]);
        face_state2(I, S, P, dir, line - 1 + s, a, 1, Vp[s]);
    }
    gauss_line2(Vm[0], Vm[1], Vm[2], Pm);
    gauss_line2(Vp[0], Vp[1], Vp[2], Pp);
    double F0[3], F1[3];
    llf2(Pm[0], Pp[0], dir, I.g, F0);
    llf2(Pm[1], Pp[1], dir, I.g, F1);
#pragma unroll
    for (int c = 0; c < 3; c++) F[c] = 0.5 * (F0[c] + F1[c]);
    hm[0] = Pm[0][0]; hm[1] = Pm[1][0];
    hp[0] = Pp[0][0]; hp[1] = Pp[1][0];
}

__device__ void face_depth2(const Inst2D &I, const Stage &S, const Pert &P, int dir, int line, int a,
                            int which, double hg[2])
{
    double V[3][3], Pq[2][3];
#pragma unroll
    for (int s = 0; s < 3; s++) face_state2(I, S, P, dir, line - 1 + s, a, which, V[s]);
    gauss_line2(V[0], V[1], V[2], Pq);
    hg[0] = Pq[0][0];
    hg[1] = Pq[1][0];
}

struct CubicW {
    double w[2][4];
    __device__ CubicW()
    {
        const double t[4] = {-1.5, -0.5, 0.5, 1.5};
        const double tg0 = -1.0 / (2.0 * sqrt(3.0));
        const double tg1 = 1.0 / (2.0 * sqrt(3.0));
#pragma unroll
        for (int q = 0; q < 2; q++) {
            const double x = q == 0 ? tg0 : tg1;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                double v = 1.0;
#pragma unroll
                for (int m = 0; m < 4; m++)
                    if (m != k) v *= (x - t[m]) / (t[k] - t[m]);
                w[q][k] = v;
            }
        }
    }
};

// Local residual R_ij of eq. (20) under perturbation P.
__device__ void local_residual2(const Inst2D &I, const Stage &S, const Pert &P, int i, int j, double R[3])
{
    double fxm[3], fxp[3], fym[3], fyp[3], dummy[2];
    double hx[4][2], hy[4][2];
    face_flux2(I, S, P, 0, j, i - 1, fxm, dummy, hx[1]);
    face_flux2(I, S, P, 0, j, i, fxp, hx[2], dummy);
    face_flux2(I, S, P, 1, i, j - 1, fym, dummy, hy[1]);
    face_flux2(I, S, P, 1, i, j, fyp, hy[2], dummy);
    face_depth2(I, S, P, 0, j, i - 2, 1, hx[0]);
    face_depth2(I, S, P, 0, j, i + 1, 0, hx[3]);
    face_depth2(I, S, P, 1, i, j - 2, 1, hy[0]);
    face_depth2(I, S, P, 1, i, j + 1, 0, hy[3]);
    const CubicW Wt;
    const double *bx = &I.bx[((long long)j * I.Nx + i) * 4];
    const double *by = &I.by[((long long)j * I.Nx + i) * 4];
    double s2 = 0.0;
#pragma unroll
    for (int be = 0; be < 2; be++)
#pragma unroll
        for (int ga = 0; ga < 2; ga++) {
            const double h = Wt.w[ga][0] * hx[0][be] + Wt.w[ga][1] * hx[1][be] + Wt.w[ga][2] * hx[2][be] + Wt.w[ga][3] * hx[3][be];
            s2 = s2 + I.g * h * bx[2 * be + ga];
        }
    double s3 = 0.0;
#pragma unroll
    for (int ga = 0; ga < 2; ga++)
#pragma unroll
        for (int be = 0; be < 2; be++) {
            const double h = Wt.w[be][0] * hy[0][ga] + Wt.w[be][1] * hy[1][ga] + Wt.w[be][2] * hy[2][ga] + Wt.w[be][3] * hy[3][ga];
            s3 = s3 + I.g * h * by[2 * be + ga];
        }
    const double S2 = -(I.dx * I.dy / 4.0) * s2;
    const double S3 = -(I.dx * I.dy / 4.0) * s3;
    R[0] = (fxp[0] - fxm[0]) / I.dx + (fyp[0] - fym[0]) / I.dy;
    R[1] = (fxp[1] - fxm[1]) / I.dx + (fyp[1] - fym[1]) / I.dy - S2 / (I.dx * I.dy);
    R[2] = (fxp[2] - fxm[2]) / I.dx + (fyp[2] - fym[2]) / I.dy - S3 / (I.dx * I.dy);
}

__device__ void stage_tile(const Inst2D &I, int i0, int j0, double *s)
{
    const int n = (int)(blockDim.x * blockDim.y);
    const int t = threadIdx.y * blockDim.x + threadIdx.x;
    for (int e = t; e < 3 * kSY * kSX; e += n) {
        const int c = e / (kSY * kSX), r = (e / kSX) % kSY, q = e % kSX;
        const int i = i0 - 2 + q, j = j0 - 2 + r;
        const bool ok = i >= 0 && i < I.Nx && j >= 0 && j < I.Ny;
        s[e] = ok ? I.U[((long long)c * I.Ny + j) * I.Nx + i] : 0.0;
    }
}

__global__ void __launch_bounds__(kTX * kTY) k_residual2d(Inst2D I, double *partial)
{
    __shared__ double s[3 * kSY * kSX];
    __shared__ double red[kTX * kTY / 64];
    const int i0 = blockIdx.x * kTX, j0 = blockIdx.y * kTY;
    stage_tile(I, i0, j0, s);
    __syncthreads();
    const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
    double n1 = 0.0;
    if (i < I.Nx && j < I.Ny) {
        const Stage S{s, i0, j0};
        const Pert P{-1000, -1000, 0, 0.0};
        double R[3];
        local_residual2(I, S, P, i, j, R);
        const long long n = (long long)I.Nx * I.Ny, cidx = (long long)j * I.Nx + i;
        I.R[cidx] = R[0];
        I.R[n + cidx] = R[1];
        I.R[2 * n + cidx] = R[2];
        n1 = fabs(R[0]) + fabs(R[1]) + fabs(R[2]);
        I.rn[cidx] = n1;
    }
    // per-tile partial sum of ||R||_1 (fixed order)
    const int t = threadIdx.y * kTX + threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) n1 += __shfl_down(n1, off, 64);
    if ((t & 63) == 0) red[t >> 6] = n1;
    __syncthreads();
    if (t == 0 && partial) {
        double sum = 0.0;
        for (int w = 0; w < kTX * kTY / 64; w++) sum += red[w];
        partial[blockIdx.y * gridDim.x + blockIdx.x] = sum;
    }
}

// sum of the tile partials in a fixed order: res = sum / (Nx Ny)
__global__ void __launch_bounds__(256) k_res2d_finalize(const double *partial, int ntiles, long long ncells,
                                                        double *res)
{
    __shared__ double red[4];
    double v = 0.0;
    for (int k = threadIdx.x; k < ntiles; k += 256) v += partial[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) *res = (red[0] + red[1] + red[2] + red[3]) / (double)ncells;
}

// Finite-difference Jacobian on the cross stencil of eq. (21), regularised per eq. (13):
// J[(b*9 + l*3 + m) * n + cell] for the blocks b of (centre, x-2, x-1, x+1, x+2, y-2, y-1, y+1,
// y+2).  Optionally the finest right-hand side (= R) and the inverse of the diagonal block.
template <typename T>
__global__ void __launch_bounds__(kTX * kTY) k_jacobian2d(Inst2D I, Perm2D Pm, T *J, T *rhs, T *Dinv)
{
    __shared__ double s[3 * kSY * kSX];
    const int i0 = blockIdx.x * kTX, j0 = blockIdx.y * kTY;
    stage_tile(I, i0, j0, s);
    __syncthreads();
    const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
    if (i >= I.Nx || j >= I.Ny) return;
    const long long n = (long long)I.Nx * I.Ny, cidx = (long long)j * I.Nx + i;
    const long long M = Pm.M, pidx = perm2d(Pm, i, j);   // output slot of this cell
    const double R0[3] = {I.R[cidx], I.R[n + cidx], I.R[2 * n + cidx]};
    const double rn = I.rn[cidx];
    if (rhs) {
        rhs[pidx] = (T)R0[0];
        rhs[M + pidx] = (T)R0[1];
        rhs[2 * M + pidx] = (T)R0[2];
    }
    const Stage S{s, i0, j0};
    const int offx[9] = {0, -2, -1, 1, 2, 0, 0, 0, 0};
    const int offy[9] = {0, 0, 0, 0, 0, -2, -1, 1, 2};
    double D[9];
    for (int b = 0; b < 9; b++) {
        const int pi = i + offx[b], pj = j + offy[b];
        const bool ok = pi >= 0 && pi < I.Nx && pj >= 0 && pj < I.Ny;
        for (int m = 0; m < 3; m++) {
            double col[3] = {0.0, 0.0, 0.0};
            if (ok) {
                const Pert P{pi, pj, m, I.eps};
                double Rp[3];
                local_residual2(I, S, P, i, j, Rp);
#pragma unroll
                for (int l = 0; l < 3; l++) col[l] = (Rp[l] - R0[l]) / I.eps;
                if (b == 0) col[m] += I.alpha * rn;
            }
#pragma unroll
            for (int l = 0; l < 3; l++) {
                J[(b * 9 + l * 3 + m) * M + pidx] = (T)col[l];
                if (b == 0) D[l * 3 + m] = col[l];
            }
        }
    }
    if (Dinv) {
        // closed-form inverse of the diagonal block (adjugate over determinant)
        const double c00 = D[4] * D[8] - D[5] * D[7];
        const double c01 = D[5] * D[6] - D[3] * D[8];
        const double c02 = D[3] * D[7] - D[4] * D[6];
        const double det = D[0] * c00 + D[1] * c01 + D[2] * c02;
        double B[9];
        B[0] = c00 / det;
        B[1] = (D[2] * D[7] - D[1] * D[8]) / det;
        B[2] = (D[1] * D[5] - D[2] * D[4]) / det;
        B[3] = c01 / det;
        B[4] = (D[0] * D[8] - D[2] * D[6]) / det;
        B[5] = (D[2] * D[3] - D[0] * D[5]) / det;
        B[6] = c02 / det;
        B[7] = (D[1] * D[6] - D[0] * D[7]) / det;
        B[8] = (D[0] * D[4] - D[1] * D[3]) / det;
#pragma unroll
        for (int e = 0; e < 9; e++) Dinv[e * M + pidx] = (T)B[e];
    }
}

// ---- launchers ---------------------------------------------------------------------------

hipError_t launch_residual2d(const Inst2D &I, double *partial, hipStream_t s)
{
    dim3 grid((I.Nx + kTX - 1) / kTX, (I.Ny + kTY - 1) / kTY);
    hipLaunchKernelGGL(k_residual2d, grid, dim3(kTX, kTY), 0, s, I, partial);
    return hipGetLastError();
}

int residual2d_tiles(int Nx, int Ny) { return ((Nx + kTX - 1) / kTX) * ((Ny + kTY - 1) / kTY); }

hipError_t launch_res2d_finalize(const double *partial, int ntiles, long long ncells, double *res,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(k_res2d_finalize, dim3(1), dim3(256), 0, s, partial, ntiles, ncells, res);
    return hipGetLastError();
}

hipError_t launch_jacobian2d(const Inst2D &I, const Perm2D &P, void *J, void *rhs, void *Dinv, int prec,
                             hipStream_t s)
{
    dim3 grid((I.Nx + kTX - 1) / kTX, (I.Ny + kTY - 1) / kTY);
    if (prec == NMG_FP32_MG)
        hipLaunchKernelGGL(k_jacobian2d<float>, grid, dim3(kTX, kTY), 0, s, I, P, (float *)J, (float *)rhs,
                           (float *)Dinv);
    else
        hipLaunchKernelGGL(k_jacobian2d<double>, grid, dim3(kTX, kTY), 0, s, I, P, (double *)J, (double *)rhs,
                           (double *)Dinv);
    return hipGetLastError();
}

}  // namespace nmg
