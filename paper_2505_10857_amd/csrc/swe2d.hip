// 2D finite-volume residual (section 4.1, eq. 20) with characteristic WENO3, Gauss quadrature
// along faces and the tensor Gauss source, and its finite-difference Jacobian on the cross
// stencil of eq. (21) (J9) or the full 21-cell stencil (J21), for gfx950.
//
// The arithmetic is that of the formulas in their printed order, without FMA contraction and
// with correctly rounded division and square root, so every face state, flux and residual is
// reproducible bit for bit; with the 1e-6 perturbation of the 2D Jacobian anything less would
// be amplified a million times.
//
// Work sharing.  The residual of cell (i, j) is assembled from 36 characteristic face states
// (x faces on rows j-1..j+1, y faces on columns i-1..i+1, both sides of the four faces of the
// cell and the inner states of the next faces out, which the source's cubics need).  A face state
// depends only on three consecutive cells of its line, so a 32x8 tile computes every face state
// its cells use once, into LDS tables, and each cell assembles its residual from them.  For the
// Jacobian a perturbation of cell p changes only the face states whose three cells include p;
// for a row at least two cells inside the grid (no ghost in its residual) and a column at a fixed
// offset of the stencil, which of the row's 36 states those are is known at compile time,
// so the interior kernel recomputes just those (at most 12) and reads the rest from the tables.
// The values equal a full re-evaluation of the perturbed local residual bit for bit.  Rows within
// two cells of a side, whose ghosts also follow the perturbed cell, take a separate kernel that
// re-evaluates all 36 face states per column.
//
// Surface variant (recon = NMG_RECON_SURFACE, template flag SURF of the state accessors): the
// reconstructions act on (eta, hu, hv), eta = h + zbar (zbar the cell average of b), in the
// characteristic basis of the two cells' (h, hu, hv); a face Gauss point's depth is eta minus b
// there; ghosts that copy a cell's depth copy its surface; each Gauss line's source takes the
// split form -g [int (eta_h - eta_ij) b_x + eta_ij (b_+ - b_-) - (b_+^2 - b_-^2) / 2].  Still
// water then has a zero residual to rounding on any bottom.
//
// Register discipline: every helper is force-inlined and passes values as small structs by
// value, indexed only by compile-time constants; boundary data of a side is selected by
// comparisons, never by a runtime array index.  The kernels keep their state in registers and
// LDS: no stack frame, no calls, no generic pointers into private memory.
#include "nmg_common.h"

namespace nmg {

constexpr int kTX = 32, kTY = 8;                       // tile of cells
constexpr int kSX = kTX + 4, kSY = kTY + 4;            // staged state (halo 2)
// face-state tables of a tile: x faces a in [i0-2, i0+kTX] on rows [j0-1, j0+kTY]; y faces
// a in [j0-2, j0+kTY] on columns [i0-1, i0+kTX]; both sides, three components
constexpr int kXA = kTX + 3, kXL = kTY + 2;
constexpr int kYA = kTY + 3, kYL = kTX + 2;
constexpr int kXS = 3 * 2 * kXL * kXA, kYS = 3 * 2 * kYL * kYA;
constexpr int kBorderNT = 64;                          // threads of a border-kernel workgroup
constexpr int kSlots = 36;                             // face states of one local residual

// Every helper is callable from host code too, so that a CPU build can replay the kernels' per-row
// arithmetic; NMG2D_CHECK is a bounds-check hook on staged and table reads for such a build.
#define NMG2D_INL __host__ __device__ __forceinline__
#ifndef NMG2D_CHECK
#define NMG2D_CHECK(cond) ((void)0)
#endif

struct V3 { double c[3]; };
struct H2 { double g[2]; };            // a depth at the two Gauss points of a face

NMG2D_INL double weno_p2(double um, double u0, double up)
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

NMG2D_INL double weno_m2(double um, double u0, double up)
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

// Characteristic WENO3 state at the face between cells a and a+1 of a line in direction DIR,
// from the three consecutive cells S0, S1, S2 of the line that its stencil uses: cells a-1..a+1
// for the minus state (W = 0, from cell a), a..a+2 for the plus state (W = 1, from cell a+1).
// The basis is the eigensystem of the face-normal flux Jacobian at the mean of cells a, a+1.
// SURF: the projection acts on the surfaces S_q.c[0] + z_q (z_q the cell average of b), the
// basis on the depths.
template <int DIR, int W, bool SURF = false>
NMG2D_INL V3 face_state_core(const V3 &S0, const V3 &S1, const V3 &S2, double g, double z0 = 0.0,
                             double z1 = 0.0, double z2 = 0.0)
{
    const V3 &Ua = W ? S0 : S1;
    const V3 &Ub = W ? S1 : S2;
    double Us[3];
#pragma unroll
    for (int c = 0; c < 3; c++) Us[c] = 0.5 * (Ua.c[c] + Ub.c[c]);
    const double h = Us[0];
    const double u = Us[1] / h;
    const double v = Us[2] / h;
    const double cc = sqrt(g * h);
    const double un = DIR == 0 ? u : v;
    const double i2c = 1.0 / (2.0 * cc);
    double L[3][3], R[3][3];
    if (DIR == 0) {
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
    double Wc[3][3], w[3];
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const V3 &Sq = q == 0 ? S0 : (q == 1 ? S1 : S2);
        const double e = SURF ? Sq.c[0] + (q == 0 ? z0 : (q == 1 ? z1 : z2)) : Sq.c[0];
#pragma unroll
        for (int f = 0; f < 3; f++)
            Wc[q][f] = L[f][0] * e + L[f][1] * Sq.c[1] + L[f][2] * Sq.c[2];
    }
#pragma unroll
    for (int f = 0; f < 3; f++)
        w[f] = W ? weno_p2(Wc[0][f], Wc[1][f], Wc[2][f]) : weno_m2(Wc[0][f], Wc[1][f], Wc[2][f]);
    V3 out;
#pragma unroll
    for (int c = 0; c < 3; c++) out.c[c] = R[c][0] * w[0] + R[c][1] * w[1] + R[c][2] * w[2];
    return out;
}

template <int DIR>
NMG2D_INL V3 flux2(const V3 &U, double g)
{
    const double h = U.c[0];
    const double u = U.c[1] / h;
    const double v = U.c[2] / h;
    V3 F;
    if (DIR == 0) {
        F.c[0] = U.c[1];
        F.c[1] = U.c[1] * u + 0.5 * g * h * h;
        F.c[2] = U.c[1] * v;
    } else {
        F.c[0] = U.c[2];
        F.c[1] = U.c[2] * u;
        F.c[2] = U.c[2] * v + 0.5 * g * h * h;
    }
    return F;
}

template <int DIR>
NMG2D_INL V3 llf2(const V3 &UL, const V3 &UR, double g)
{
    const V3 FL = flux2<DIR>(UL, g);
    const V3 FR = flux2<DIR>(UR, g);
    const double unL = UL.c[1 + DIR] / UL.c[0], unR = UR.c[1 + DIR] / UR.c[0];
    const double sL = fabs(unL) + sqrt(g * UL.c[0]);
    const double sR = fabs(unR) + sqrt(g * UR.c[0]);
    const double a = sL > sR ? sL : sR;
    V3 F;
#pragma unroll
    for (int c = 0; c < 3; c++) F.c[c] = 0.5 * (FL.c[c] + FR.c[c] - a * (UR.c[c] - UL.c[c]));
    return F;
}

// The quadratic through three face averages at the Gauss point G (0: lower, 1: upper) of the
// face (its curvature term is zero there): V0 + t (Vp - Vm) / 2, t = -+1/(2 sqrt 3).
template <int G>
NMG2D_INL V3 gauss_pt2(const V3 &Vm, const V3 &V0, const V3 &Vp)
{
    const double t = G == 0 ? -1.0 / (2.0 * sqrt(3.0)) : 1.0 / (2.0 * sqrt(3.0));
    V3 P;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const double slope = (Vp.c[c] - Vm.c[c]) * 0.5;
        P.c[c] = V0.c[c] + t * slope;
    }
    return P;
}

// Lagrange weight of node K (nodes -3/2, -1/2, 1/2, 3/2) of the cubic at the Gauss point Q
// (0: -1/(2 sqrt 3), 1: +1/(2 sqrt 3)), as the product over the other nodes in node order
template <int Q, int K>
NMG2D_INL double cubic_w2()
{
    const double x = Q == 0 ? -1.0 / (2.0 * sqrt(3.0)) : 1.0 / (2.0 * sqrt(3.0));
    const double t[4] = {-1.5, -0.5, 0.5, 1.5};
    double v = 1.0;
#pragma unroll
    for (int m = 0; m < 4; m++)
        if (m != K) v *= (x - t[m]) / (t[K] - t[m]);
    return v;
}

template <int Q>
NMG2D_INL double cubic_at2(double h0, double h1, double h2, double h3)
{
    return cubic_w2<Q, 0>() * h0 + cubic_w2<Q, 1>() * h1 + cubic_w2<Q, 2>() * h2 + cubic_w2<Q, 3>() * h3;
}

// Local residual R_ij of eq. (20) from its 36 face states.  FS::get<DIR, W, K, A>() gives the
// state of side W of the face between cells A and A+1 (relative to the row cell along the
// direction DIR) on the line at offset K across it.  bx, by: the cell's bottom slopes at its 2x2
// Gauss points ([beta][gamma], beta the y point).
// hm, hp: the first component of the two states at the Gauss points (the depth, or the surface
// in the surface variant, whose depths are then those minus b0, b1, b at the two points)
template <int DIR, int A, class FS>
NMG2D_INL V3 face_flux_at(const FS &fs, double g, H2 &hm, H2 &hp, double b0 = 0.0, double b1 = 0.0)
{
    const V3 Vm0 = fs.template get<DIR, 0, -1, A>(), Vm1 = fs.template get<DIR, 0, 0, A>(),
             Vm2 = fs.template get<DIR, 0, 1, A>();
    const V3 Vp0 = fs.template get<DIR, 1, -1, A>(), Vp1 = fs.template get<DIR, 1, 0, A>(),
             Vp2 = fs.template get<DIR, 1, 1, A>();
    V3 Pm0 = gauss_pt2<0>(Vm0, Vm1, Vm2), Pm1 = gauss_pt2<1>(Vm0, Vm1, Vm2);
    V3 Pp0 = gauss_pt2<0>(Vp0, Vp1, Vp2), Pp1 = gauss_pt2<1>(Vp0, Vp1, Vp2);
    hm.g[0] = Pm0.c[0]; hm.g[1] = Pm1.c[0];
    hp.g[0] = Pp0.c[0]; hp.g[1] = Pp1.c[0];
    if constexpr (FS::surf) {
        Pm0.c[0] = Pm0.c[0] - b0; Pp0.c[0] = Pp0.c[0] - b0;
        Pm1.c[0] = Pm1.c[0] - b1; Pp1.c[0] = Pp1.c[0] - b1;
    }
    const V3 F0 = llf2<DIR>(Pm0, Pp0, g);
    const V3 F1 = llf2<DIR>(Pm1, Pp1, g);
    V3 F;
#pragma unroll
    for (int c = 0; c < 3; c++) F.c[c] = 0.5 * (F0.c[c] + F1.c[c]);
    return F;
}

template <int DIR, int W, int A, class FS>
NMG2D_INL H2 face_depth_at(const FS &fs)
{
    const V3 V0 = fs.template get<DIR, W, -1, A>(), V1 = fs.template get<DIR, W, 0, A>(),
             V2 = fs.template get<DIR, W, 1, A>();
    H2 hg;
    hg.g[0] = gauss_pt2<0>(V0, V1, V2).c[0];
    hg.g[1] = gauss_pt2<1>(V0, V1, V2).c[0];
    return hg;
}

// (i, j): the row cell; h_own: its depth (perturbed when the column perturbs it), which the
// surface variant's source needs.
template <class FS>
NMG2D_INL V3 assemble_residual(const FS &fs, const Inst2D &I, const double bx[4], const double by[4], int i = 0,
                               int j = 0, double h_own = 0.0)
{
    H2 hx0, hx1, hx2, hx3, hy0, hy1, hy2, hy3, dum;
    // b at the Gauss points of the cell's four faces (surface variant)
    double bxm0 = 0.0, bxm1 = 0.0, bxp0 = 0.0, bxp1 = 0.0, bym0 = 0.0, bym1 = 0.0, byp0 = 0.0, byp1 = 0.0;
    if constexpr (FS::surf) {
        const long long fx = ((long long)j * (I.Nx + 1) + i) * 2, fy = ((long long)j * I.Nx + i) * 2;
        bxm0 = I.zfx[fx]; bxm1 = I.zfx[fx + 1]; bxp0 = I.zfx[fx + 2]; bxp1 = I.zfx[fx + 3];
        bym0 = I.zfy[fy]; bym1 = I.zfy[fy + 1];
        byp0 = I.zfy[fy + 2 * I.Nx]; byp1 = I.zfy[fy + 2 * I.Nx + 1];
    }
    const V3 fxm = face_flux_at<0, -1>(fs, I.g, dum, hx1, bxm0, bxm1);    // x_{i-1/2}: plus state from cell i
    const V3 fxp = face_flux_at<0, 0>(fs, I.g, hx2, dum, bxp0, bxp1);     // x_{i+1/2}: minus state from cell i
    const V3 fym = face_flux_at<1, -1>(fs, I.g, dum, hy1, bym0, bym1);
    const V3 fyp = face_flux_at<1, 0>(fs, I.g, hy2, dum, byp0, byp1);
    hx0 = face_depth_at<0, 1, -2>(fs);                        // x_{i-3/2}: plus state, cell i-1
    hx3 = face_depth_at<0, 0, 1>(fs);                         // x_{i+3/2}: minus state, cell i+1
    hy0 = face_depth_at<1, 1, -2>(fs);
    hy3 = face_depth_at<1, 0, 1>(fs);
    // the surface variant integrates (eta_h - eta_ij) b_x by Gauss points and the rest exactly
    double eta = 0.0;
    if constexpr (FS::surf) eta = h_own + I.zavg[((long long)j + 2) * (I.Nx + 4) + i + 2];
    // S2: the cubic in x along each y Gauss line beta at the x Gauss points gamma
    double s2 = 0.0;
#pragma unroll
    for (int be = 0; be < 2; be++) {
        const double h0 = cubic_at2<0>(hx0.g[be], hx1.g[be], hx2.g[be], hx3.g[be]);
        s2 = s2 + I.g * (FS::surf ? h0 - eta : h0) * bx[2 * be + 0];
        const double h1 = cubic_at2<1>(hx0.g[be], hx1.g[be], hx2.g[be], hx3.g[be]);
        s2 = s2 + I.g * (FS::surf ? h1 - eta : h1) * bx[2 * be + 1];
    }
    // S3: the cubic in y along each x Gauss line gamma at the y Gauss points beta
    double s3 = 0.0;
#pragma unroll
    for (int ga = 0; ga < 2; ga++) {
        const double h0 = cubic_at2<0>(hy0.g[ga], hy1.g[ga], hy2.g[ga], hy3.g[ga]);
        s3 = s3 + I.g * (FS::surf ? h0 - eta : h0) * by[0 + ga];
        const double h1 = cubic_at2<1>(hy0.g[ga], hy1.g[ga], hy2.g[ga], hy3.g[ga]);
        s3 = s3 + I.g * (FS::surf ? h1 - eta : h1) * by[2 + ga];
    }
    double S2 = -(I.dx * I.dy / 4.0) * s2;
    double S3 = -(I.dx * I.dy / 4.0) * s3;
    if constexpr (FS::surf) {
        double e2 = 0.0;
        e2 = e2 + I.g * (eta * (bxp0 - bxm0) - (bxp0 * bxp0 - bxm0 * bxm0) / 2.0);
        e2 = e2 + I.g * (eta * (bxp1 - bxm1) - (bxp1 * bxp1 - bxm1 * bxm1) / 2.0);
        double e3 = 0.0;
        e3 = e3 + I.g * (eta * (byp0 - bym0) - (byp0 * byp0 - bym0 * bym0) / 2.0);
        e3 = e3 + I.g * (eta * (byp1 - bym1) - (byp1 * byp1 - bym1 * bym1) / 2.0);
        S2 = -(I.dx * I.dy / 4.0) * s2 - (I.dy / 2.0) * e2;
        S3 = -(I.dx * I.dy / 4.0) * s3 - (I.dx / 2.0) * e3;
    }
    V3 R;
    R.c[0] = (fxp.c[0] - fxm.c[0]) / I.dx + (fyp.c[0] - fym.c[0]) / I.dy;
    R.c[1] = (fxp.c[1] - fxm.c[1]) / I.dx + (fyp.c[1] - fym.c[1]) / I.dy - S2 / (I.dx * I.dy);
    R.c[2] = (fxp.c[2] - fxm.c[2]) / I.dx + (fyp.c[2] - fym.c[2]) / I.dy - S3 / (I.dx * I.dy);
    return R;
}

// ---- ghost cells ---------------------------------------------------------------------------

// the value of side k (0 left, 1 right, 2 bottom, 3 top) out of four scalars
NMG2D_INL double side4(int k, double a0, double a1, double a2, double a3)
{
    return k == 0 ? a0 : (k == 1 ? a1 : (k == 2 ? a2 : a3));
}

// state in LDS: s[c][y][x] for cells (i0 - 2 + x, j0 - 2 + y); SURF: z[y][x], the cell averages
// of b of the same cells (ghosts included)
template <bool SURF>
struct LdsStateT {
    static constexpr bool surf = SURF;
    const double *s, *z;
    int i0, j0;
    NMG2D_INL double operator()(int c, int i, int j) const
    {
        NMG2D_CHECK(c >= 0 && c < 3 && j - j0 + 2 >= 0 && j - j0 + 2 < kSY && i - i0 + 2 >= 0 && i - i0 + 2 < kSX);
        return s[(c * kSY + (j - j0 + 2)) * kSX + (i - i0 + 2)];
    }
    NMG2D_INL double zb(int i, int j) const
    {
        NMG2D_CHECK(j - j0 + 2 >= 0 && j - j0 + 2 < kSY && i - i0 + 2 >= 0 && i - i0 + 2 < kSX);
        return z[(j - j0 + 2) * kSX + (i - i0 + 2)];
    }
};
using LdsState = LdsStateT<false>;

// state in global memory [3][Ny][Nx]; SURF: zavg [Ny+4][Nx+4] (cells -2..Nx+1 x -2..Ny+1)
template <bool SURF>
struct GlobalStateT {
    static constexpr bool surf = SURF;
    const double *U, *zavg;
    int Nx, Ny;
    NMG2D_INL double operator()(int c, int i, int j) const
    {
        NMG2D_CHECK(c >= 0 && c < 3 && i >= 0 && i < Nx && j >= 0 && j < Ny);
        return U[((long long)c * Ny + j) * Nx + i];
    }
    NMG2D_INL double zb(int i, int j) const
    {
        NMG2D_CHECK(i >= -2 && i < Nx + 2 && j >= -2 && j < Ny + 2);
        return zavg[((long long)j + 2) * (Nx + 4) + i + 2];
    }
};

// Cell (i, j), ghosts included (y sides first, then x sides), with component pm of the interior
// cell (pi, pj) raised by eps; a ghost built from that cell follows it.
template <class ST>
NMG2D_INL V3 cell2(const Inst2D &I, const ST &st, int i, int j, int pi, int pj, int pm, double eps)
{
    int ii = i, jj = j, flip_u = 0, flip_v = 0, state = -1, set_h = -1, set_q = -1;
    if (j < 0 || j >= I.Ny) {
        const int side = j < 0 ? 2 : 3;
        int kind = j < 0 ? I.bc_kind[2] : I.bc_kind[3];
        if (side == 2 && I.bc_kind[2] == NMG_BC_WALL && I.wall_x > I.x0) {
            const double xc = I.x0 + (i + 0.5) * I.dx;
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
        const int kind = i < 0 ? I.bc_kind[0] : I.bc_kind[1];
        const int b = i < 0 ? 0 : I.Nx - 1;
        const int m = i < 0 ? -1 - i : 2 * I.Nx - 1 - i;
        ii = b;
        if (kind == NMG_BC_WALL) { ii = m; flip_u = 1; }
        else if (kind == NMG_BC_STATE) state = side;
        else if (kind == NMG_BC_DISCHARGE) set_q = side;
        else if (kind == NMG_BC_DEPTH) set_h = side;
    }
    V3 out;
    if (state >= 0) {
        const double h = side4(state, I.bc_h[0], I.bc_h[1], I.bc_h[2], I.bc_h[3]);
        out.c[0] = h;
        out.c[1] = h * side4(state, I.bc_u[0], I.bc_u[1], I.bc_u[2], I.bc_u[3]);
        out.c[2] = h * side4(state, I.bc_v[0], I.bc_v[1], I.bc_v[2], I.bc_v[3]);
        return out;
    }
    const bool hit = ii == pi && jj == pj;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const double x = st(c, ii, jj);
        out.c[c] = (hit && c == pm) ? x + eps : x;
    }
    if (flip_u) out.c[1] = -out.c[1];
    if (flip_v) out.c[2] = -out.c[2];
    if constexpr (ST::surf)      // a ghost that copies a depth copies the surface
        if (ii != i || jj != j) out.c[0] = out.c[0] + st.zb(ii, jj) - st.zb(i, j);
    if (set_h >= 0) out.c[0] = side4(set_h, I.bc_h[0], I.bc_h[1], I.bc_h[2], I.bc_h[3]);
    if (set_q >= 0) {
        const double q = side4(set_q, I.bc_q[0], I.bc_q[1], I.bc_q[2], I.bc_q[3]);
        if (set_q < 2) out.c[1] = q;
        else out.c[2] = q;
    }
    return out;
}

// face state of side W of face a (between cells a, a+1) on line k in direction DIR, any
// position within two cells of the grid, ghosts applied, under the perturbation (pi, pj, pm)
template <int DIR, int W, class ST>
NMG2D_INL V3 face_state_general(const Inst2D &I, const ST &st, int k, int a, int pi, int pj, int pm, double eps)
{
    V3 S[3];
    double z[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const int t = a - 1 + W + q;
        S[q] = DIR == 0 ? cell2(I, st, t, k, pi, pj, pm, eps) : cell2(I, st, k, t, pi, pj, pm, eps);
        if constexpr (ST::surf) z[q] = DIR == 0 ? st.zb(t, k) : st.zb(k, t);
    }
    return face_state_core<DIR, W, ST::surf>(S[0], S[1], S[2], I.g, z[0], z[1], z[2]);
}

// ---- face-state tables of a tile ----------------------------------------------------------

NMG2D_INL int xs_index(int c, int w, int line, int a)   // line, a relative to the table origin
{
    NMG2D_CHECK(line >= 0 && line < kXL && a >= (w ? 0 : 1) && a < kXA - (w ? 1 : 0));
    return ((c * 2 + w) * kXL + line) * kXA + a;
}
NMG2D_INL int ys_index(int c, int w, int line, int a)
{
    NMG2D_CHECK(line >= 0 && line < kYL && a >= (w ? 0 : 1) && a < kYA - (w ? 1 : 0));
    return ((c * 2 + w) * kYL + line) * kYA + a;
}

// thread t of n stages its share of the tile's state (and, for the surface variant, the cell
// averages of b of the same cells, ghosts included, into z)
NMG2D_INL void stage_tile(const Inst2D &I, int i0, int j0, double *s, int t, int n, double *z = nullptr)
{
    for (int e = t; e < 3 * kSY * kSX; e += n) {
        const int c = e / (kSY * kSX), r = (e / kSX) % kSY, q = e % kSX;
        const int i = i0 - 2 + q, j = j0 - 2 + r;
        const bool ok = i >= 0 && i < I.Nx && j >= 0 && j < I.Ny;
        s[e] = ok ? I.U[((long long)c * I.Ny + j) * I.Nx + i] : 0.0;
    }
    if (z)
        for (int e = t; e < kSY * kSX; e += n) {
            const int r = e / kSX, q = e % kSX;
            const int i = i0 - 2 + q, j = j0 - 2 + r;
            const bool ok = i >= -2 && i < I.Nx + 2 && j >= -2 && j < I.Ny + 2;
            z[e] = ok ? I.zavg[((long long)j + 2) * (I.Nx + 4) + i + 2] : 0.0;
        }
}

// every face state the tile's cells use, unperturbed (after stage_tile and a barrier): the minus
// states (W = 0) of faces i0-1 .. i0+kTX, the plus states (W = 1) of faces i0-2 .. i0+kTX-1 (and
// the same along y), whose three cells all lie in the staged region
template <int W, class ST>
NMG2D_INL void face_tables_side(const Inst2D &I, const ST &st, double *xs, double *ys, int t, int n)
{
    constexpr int xa = kXA - 1, ya = kYA - 1;      // faces per line used on this side
    for (int e = t; e < kXL * xa; e += n) {
        const int line = e / xa, a = e - line * xa + (W ? 0 : 1);
        const V3 v = face_state_general<0, W>(I, st, st.j0 - 1 + line, st.i0 - 2 + a, -1000, -1000, 0, 0.0);
#pragma unroll
        for (int c = 0; c < 3; c++) xs[xs_index(c, W, line, a)] = v.c[c];
    }
    for (int e = t; e < kYL * ya; e += n) {
        const int line = e / ya, a = e - line * ya + (W ? 0 : 1);
        const V3 v = face_state_general<1, W>(I, st, st.i0 - 1 + line, st.j0 - 2 + a, -1000, -1000, 0, 0.0);
#pragma unroll
        for (int c = 0; c < 3; c++) ys[ys_index(c, W, line, a)] = v.c[c];
    }
}

template <class ST>
NMG2D_INL void face_tables(const Inst2D &I, const ST &st, double *xs, double *ys, int t, int n)
{
    face_tables_side<0>(I, st, xs, ys, t, n);
    face_tables_side<1>(I, st, xs, ys, t, n);
}

// face states of the row cell (i, j) read from the tables
template <bool SURF>
struct TableFS {
    static constexpr bool surf = SURF;
    const double *xs, *ys;
    int xi, xj;        // the row cell relative to the tables' origins: i - i0, j - j0
    template <int DIR, int W, int K, int A>
    NMG2D_INL V3 get() const
    {
        V3 v;
#pragma unroll
        for (int c = 0; c < 3; c++)
            v.c[c] = DIR == 0 ? xs[xs_index(c, W, xj + 1 + K, xi + 2 + A)]
                              : ys[ys_index(c, W, xi + 1 + K, xj + 2 + A)];
        return v;
    }
};

// Face states of an interior row cell under a perturbation of component pm of the cell at the
// offset (DX, DY) of the cross stencil: a state whose three cells include that cell is
// recomputed from the staged state, every other one read from the tables.
template <int DX, int DY, bool SURF>
struct PerturbedFS {
    static constexpr bool surf = SURF;
    TableFS<SURF> tab;
    LdsStateT<SURF> st;
    int i, j, pm;
    double eps, g;

    template <int DIR, int W, int K, int A>
    static constexpr bool hit()
    {
        // along the line the state uses cells A-1+W .. A+1+W; the line sits at offset K across
        return DIR == 0 ? (K == DY && DX >= A - 1 + W && DX <= A + 1 + W)
                        : (K == DX && DY >= A - 1 + W && DY <= A + 1 + W);
    }

    template <int DIR, int W, int K, int A, int Q>
    NMG2D_INL V3 cell() const
    {
        constexpr int t = A - 1 + W + Q;                       // along the line
        constexpr int ci = DIR == 0 ? t : K, cj = DIR == 0 ? K : t;
        constexpr bool on = ci == DX && cj == DY;
        V3 v;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const double x = st(c, i + ci, j + cj);
            v.c[c] = (on && c == pm) ? x + eps : x;
        }
        return v;
    }

    template <int DIR, int W, int K, int A>
    NMG2D_INL V3 get() const
    {
        if constexpr (hit<DIR, W, K, A>()) {
            constexpr int t0 = A - 1 + W;
            double z0 = 0.0, z1 = 0.0, z2 = 0.0;
            if constexpr (SURF) {
                z0 = DIR == 0 ? st.zb(i + t0, j + K) : st.zb(i + K, j + t0);
                z1 = DIR == 0 ? st.zb(i + t0 + 1, j + K) : st.zb(i + K, j + t0 + 1);
                z2 = DIR == 0 ? st.zb(i + t0 + 2, j + K) : st.zb(i + K, j + t0 + 2);
            }
            return face_state_core<DIR, W, SURF>(cell<DIR, W, K, A, 0>(), cell<DIR, W, K, A, 1>(),
                                                 cell<DIR, W, K, A, 2>(), g, z0, z1, z2);
        } else {
            return tab.template get<DIR, W, K, A>();
        }
    }
};

// ---- residual -------------------------------------------------------------------------------

NMG2D_INL void load_slopes(const Inst2D &I, int i, int j, double bx[4], double by[4])
{
    const long long g = ((long long)j * I.Nx + i) * 4;
#pragma unroll
    for (int e = 0; e < 4; e++) {
        bx[e] = I.bx[g + e];
        by[e] = I.by[g + e];
    }
}

template <bool SURF>
__global__ void __launch_bounds__(kTX * kTY) k_residual2d(Inst2D I, double *partial)
{
    __shared__ double s[3 * kSY * kSX];
    __shared__ double zs[SURF ? kSY * kSX : 1];
    __shared__ double xs[kXS], ys[kYS];
    __shared__ double red[kTX * kTY / 64];
    const int i0 = blockIdx.x * kTX, j0 = blockIdx.y * kTY;
    const int tid = threadIdx.y * kTX + threadIdx.x;
    stage_tile(I, i0, j0, s, tid, kTX * kTY, SURF ? zs : nullptr);
    __syncthreads();
    const LdsStateT<SURF> st{s, zs, i0, j0};
    face_tables(I, st, xs, ys, tid, kTX * kTY);
    __syncthreads();
    const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
    double n1 = 0.0;
    if (i < I.Nx && j < I.Ny) {
        double bx[4], by[4];
        load_slopes(I, i, j, bx, by);
        const TableFS<SURF> fs{xs, ys, i - i0, j - j0};
        const V3 R = assemble_residual(fs, I, bx, by, i, j, st(0, i, j));
        const long long n = (long long)I.Nx * I.Ny, cidx = (long long)j * I.Nx + i;
        I.R[cidx] = R.c[0];
        I.R[n + cidx] = R.c[1];
        I.R[2 * n + cidx] = R.c[2];
        n1 = fabs(R.c[0]) + fabs(R.c[1]) + fabs(R.c[2]);
        I.rn[cidx] = n1;
    }
    // per-tile partial sum of ||R||_1 (fixed order)
    const int t = threadIdx.y * kTX + threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) n1 += __shfl_down(n1, off, 64);
    if ((t & 63) == 0) red[t >> 6] = n1;
    __syncthreads();
    if (t == 0 && partial) {
        double sum = 0.0;
#pragma unroll
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

// ---- Jacobian -------------------------------------------------------------------------------

// Block b of the cross stencil of eq. (21): centre, x-2, x-1, x+1, x+2, y-2, y-1, y+1, y+2.
// Output: J[(b*9 + l*3 + m) * M + slot], the column (b, m) of row l, in the cell order Pm.
struct JacOut {
    long long M, slot;
    double R0, R1, R2, rn, alpha, eps;
};

template <typename T>
NMG2D_INL void store_column(T *J, const JacOut &o, int b, int m, const V3 &Rp, double d[3])
{
    double c0 = (Rp.c[0] - o.R0) / o.eps;
    double c1 = (Rp.c[1] - o.R1) / o.eps;
    double c2 = (Rp.c[2] - o.R2) / o.eps;
    if (b == 0) {
        if (m == 0) c0 += o.alpha * o.rn;
        else if (m == 1) c1 += o.alpha * o.rn;
        else c2 += o.alpha * o.rn;
    }
    J[(b * 9 + 0 * 3 + m) * o.M + o.slot] = (T)c0;
    J[(b * 9 + 1 * 3 + m) * o.M + o.slot] = (T)c1;
    J[(b * 9 + 2 * 3 + m) * o.M + o.slot] = (T)c2;
    d[0] = c0; d[1] = c1; d[2] = c2;
}

template <typename T>
NMG2D_INL void store_zero_column(T *J, const JacOut &o, int b, int m)
{
#pragma unroll
    for (int l = 0; l < 3; l++) J[(b * 9 + l * 3 + m) * o.M + o.slot] = (T)0.0;
}

// inverse of the diagonal block D (row-major d[l*3+m]) by the adjugate over the determinant
template <typename T>
NMG2D_INL void store_dinv(T *Dinv, long long M, long long slot, const double D[9])
{
    const double c00 = D[4] * D[8] - D[5] * D[7];
    const double c01 = D[5] * D[6] - D[3] * D[8];
    const double c02 = D[3] * D[7] - D[4] * D[6];
    const double det = D[0] * c00 + D[1] * c01 + D[2] * c02;
    Dinv[0 * M + slot] = (T)(c00 / det);
    Dinv[1 * M + slot] = (T)((D[2] * D[7] - D[1] * D[8]) / det);
    Dinv[2 * M + slot] = (T)((D[1] * D[5] - D[2] * D[4]) / det);
    Dinv[3 * M + slot] = (T)(c01 / det);
    Dinv[4 * M + slot] = (T)((D[0] * D[8] - D[2] * D[6]) / det);
    Dinv[5 * M + slot] = (T)((D[2] * D[3] - D[0] * D[5]) / det);
    Dinv[6 * M + slot] = (T)(c02 / det);
    Dinv[7 * M + slot] = (T)((D[1] * D[6] - D[0] * D[7]) / det);
    Dinv[8 * M + slot] = (T)((D[0] * D[4] - D[1] * D[3]) / det);
}

// a row whose residual involves a ghost cell: within two cells of a side
NMG2D_INL bool border_row(const Inst2D &I, int i, int j)
{
    return i < 2 || j < 2 || i >= I.Nx - 2 || j >= I.Ny - 2;
}

template <int B, typename T, bool SURF>
NMG2D_INL void interior_column(T *J, const JacOut &o, const TableFS<SURF> &tab, const LdsStateT<SURF> &st,
                               const Inst2D &I, int i, int j, int m, const double bx[4], const double by[4],
                               double d[3])
{
    const PerturbedFS<stencil_dx(21, B), stencil_dy(21, B), SURF> fs{tab, st, i, j, m, I.eps, I.g};
    double h_own = 0.0;
    if constexpr (SURF) {
        const double x = st(0, i, j);
        h_own = (B == 0 && m == 0) ? x + I.eps : x;
    }
    const V3 Rp = assemble_residual(fs, I, bx, by, i, j, h_own);
    store_column(J, o, B, m, Rp, d);
}

// the 3 NB columns of the interior row (i, j) of a tile whose state and face tables are staged
// (the first nine blocks of the full stencil are the cross, so one offset table serves both)
template <typename T, int NB, bool SURF>
NMG2D_INL void jacobian_interior_row(const Inst2D &I, const Perm2D &Pm, T *J, T *rhs, T *Dinv, const double *xs,
                                     const double *ys, const LdsStateT<SURF> &st, int i, int j)
{
    const int i0 = st.i0, j0 = st.j0;
    const long long n = (long long)I.Nx * I.Ny, cidx = (long long)j * I.Nx + i;
    JacOut o;
    o.M = Pm.M;
    o.slot = perm2d(Pm, i, j);
    o.R0 = I.R[cidx];
    o.R1 = I.R[n + cidx];
    o.R2 = I.R[2 * n + cidx];
    o.rn = I.rn[cidx];
    o.alpha = I.alpha;
    o.eps = I.eps;
    if (rhs) {
        rhs[o.slot] = (T)o.R0;
        rhs[o.M + o.slot] = (T)o.R1;
        rhs[2 * o.M + o.slot] = (T)o.R2;
    }
    double bx[4], by[4];
    load_slopes(I, i, j, bx, by);
    const TableFS<SURF> tab{xs, ys, i - i0, j - j0};
    double D[9];
#pragma unroll
    for (int e = 0; e < 9; e++) D[e] = 0.0;
    // one column at a time (a rolled loop over the columns, the stencil offset dispatched to
    // its compile-time form), so that only one column's values are live
#pragma unroll 1
    for (int col = 0; col < 3 * NB; col++) {
        const int b = col / 3, m = col - 3 * b;
        double d[3];
        switch (b) {
        case 0: interior_column<0>(J, o, tab, st, I, i, j, m, bx, by, d); break;
        case 1: interior_column<1>(J, o, tab, st, I, i, j, m, bx, by, d); break;
        case 2: interior_column<2>(J, o, tab, st, I, i, j, m, bx, by, d); break;
        case 3: interior_column<3>(J, o, tab, st, I, i, j, m, bx, by, d); break;
        case 4: interior_column<4>(J, o, tab, st, I, i, j, m, bx, by, d); break;
        case 5: interior_column<5>(J, o, tab, st, I, i, j, m, bx, by, d); break;
        case 6: interior_column<6>(J, o, tab, st, I, i, j, m, bx, by, d); break;
        case 7: interior_column<7>(J, o, tab, st, I, i, j, m, bx, by, d); break;
        case 8: interior_column<8>(J, o, tab, st, I, i, j, m, bx, by, d); break;
        default:
            if constexpr (NB == 21) {
                switch (b) {
                case 9: interior_column<9>(J, o, tab, st, I, i, j, m, bx, by, d); break;
                case 10: interior_column<10>(J, o, tab, st, I, i, j, m, bx, by, d); break;
                case 11: interior_column<11>(J, o, tab, st, I, i, j, m, bx, by, d); break;
                case 12: interior_column<12>(J, o, tab, st, I, i, j, m, bx, by, d); break;
                case 13: interior_column<13>(J, o, tab, st, I, i, j, m, bx, by, d); break;
                case 14: interior_column<14>(J, o, tab, st, I, i, j, m, bx, by, d); break;
                case 15: interior_column<15>(J, o, tab, st, I, i, j, m, bx, by, d); break;
                case 16: interior_column<16>(J, o, tab, st, I, i, j, m, bx, by, d); break;
                case 17: interior_column<17>(J, o, tab, st, I, i, j, m, bx, by, d); break;
                case 18: interior_column<18>(J, o, tab, st, I, i, j, m, bx, by, d); break;
                case 19: interior_column<19>(J, o, tab, st, I, i, j, m, bx, by, d); break;
                default: interior_column<20>(J, o, tab, st, I, i, j, m, bx, by, d); break;
                }
            }
            break;
        }
        if (b == 0) {
            if (m == 0) { D[0] = d[0]; D[3] = d[1]; D[6] = d[2]; }
            else if (m == 1) { D[1] = d[0]; D[4] = d[1]; D[7] = d[2]; }
            else { D[2] = d[0]; D[5] = d[1]; D[8] = d[2]; }
        }
    }
    if (Dinv) store_dinv(Dinv, o.M, o.slot, D);
}

// Finite-difference Jacobian (eq. 12, 13) of the rows at least two cells inside the grid, one
// thread per row: for each component m, the NB columns of the stencil.  Optionally the finest
// right-hand side (= R) and the inverse of the diagonal block.
template <typename T, int NB, bool SURF>
__global__ void __launch_bounds__(kTX * kTY) k_jacobian2d(Inst2D I, Perm2D Pm, T *J, T *rhs, T *Dinv)
{
    __shared__ double s[3 * kSY * kSX];
    __shared__ double zs[SURF ? kSY * kSX : 1];
    __shared__ double xs[kXS], ys[kYS];
    const int i0 = blockIdx.x * kTX, j0 = blockIdx.y * kTY;
    const int tid = threadIdx.y * kTX + threadIdx.x;
    stage_tile(I, i0, j0, s, tid, kTX * kTY, SURF ? zs : nullptr);
    __syncthreads();
    const LdsStateT<SURF> st{s, zs, i0, j0};
    face_tables(I, st, xs, ys, tid, kTX * kTY);
    __syncthreads();
    const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
    if (i >= I.Nx || j >= I.Ny || border_row(I, i, j)) return;
    jacobian_interior_row<T, NB, SURF>(I, Pm, J, rhs, Dinv, xs, ys, st, i, j);
}

// Face states of a border row, full re-evaluation: the 36 states sit in per-thread LDS slots,
// slot q at slots[(q*3 + c) * kBorderNT + lane].
template <bool SURF>
struct SlotFS {
    static constexpr bool surf = SURF;
    const double *slots;
    int lane;
    // slot of a face state: per direction 18, in the order A = -1 (6: W, K), A = 0 (6),
    // A = -2 (3: K, plus side), A = 1 (3: K, minus side)
    template <int DIR, int W, int K, int A>
    static constexpr int slot()
    {
        return DIR * 18 + (A == -1 ? (W * 3 + K + 1) : A == 0 ? 6 + W * 3 + K + 1 : A == -2 ? 12 + K + 1 : 15 + K + 1);
    }
    template <int DIR, int W, int K, int A>
    NMG2D_INL V3 get() const
    {
        constexpr int q = slot<DIR, W, K, A>();
        V3 v;
#pragma unroll
        for (int c = 0; c < 3; c++) v.c[c] = slots[(q * 3 + c) * kBorderNT + lane];
        return v;
    }
};

// the face state of slot q of row (i, j) under a perturbation (runtime slot decode)
template <class ST>
NMG2D_INL V3 slot_state(const Inst2D &I, const ST &st, int q, int i, int j, int pi, int pj, int pm, double eps)
{
    const int dir = q / 18, r = q - 18 * dir;
    int w, K, A;
    if (r < 6) { A = -1; w = r / 3; K = r % 3 - 1; }
    else if (r < 12) { A = 0; w = (r - 6) / 3; K = (r - 6) % 3 - 1; }
    else if (r < 15) { A = -2; w = 1; K = r - 13; }
    else { A = 1; w = 0; K = r - 16; }
    if (dir == 0) {
        const int k = j + K, a = i + A;
        return w ? face_state_general<0, 1>(I, st, k, a, pi, pj, pm, eps)
                 : face_state_general<0, 0>(I, st, k, a, pi, pj, pm, eps);
    }
    const int k = i + K, a = j + A;
    return w ? face_state_general<1, 1>(I, st, k, a, pi, pj, pm, eps)
             : face_state_general<1, 0>(I, st, k, a, pi, pj, pm, eps);
}

// the cell of border row number r (rows within two cells of a side, bottom band, top band, then
// the two side bands of the rows in between)
NMG2D_INL void border_cell(const Inst2D &I, long long r, int &i, int &j)
{
    const int nb = I.Ny < 2 ? I.Ny : 2;                 // bottom band rows
    const int jt = I.Ny - 2 > nb ? I.Ny - 2 : nb;       // first top band row
    const long long bottom = (long long)nb * I.Nx, top = (long long)(I.Ny - jt) * I.Nx;
    if (r < bottom) { j = (int)(r / I.Nx); i = (int)(r - (long long)j * I.Nx); return; }
    r -= bottom;
    if (r < top) { j = jt + (int)(r / I.Nx); i = (int)(r - (long long)(j - jt) * I.Nx); return; }
    r -= top;
    const int side = I.Nx < 4 ? I.Nx : 4;                // side cells per middle row
    j = nb + (int)(r / side);
    const int k = (int)(r - (long long)(j - nb) * side);
    i = (I.Nx <= 4 || k < 2) ? k : I.Nx - 4 + k;
}

long long border_rows2d(int Nx, int Ny)
{
    const long long inner = (long long)(Nx > 4 ? Nx - 4 : 0) * (Ny > 4 ? Ny - 4 : 0);
    return (long long)Nx * Ny - inner;
}

// column col (b*3 + m) of border row number r, its face states in the slot array at lane `lane`
// (stride kBorderNT); d: the column's FP64 values.  Returns the row's output slot.
template <typename T, bool SURF>
NMG2D_INL long long jacobian_border_column(const Inst2D &I, const Perm2D &Pm, T *J, T *rhs, double *slots, int lane,
                                           long long r, int col, double d[3])
{
    const int b = col / 3, m = col - 3 * b;
    int i, j;
    border_cell(I, r, i, j);
    const long long n = (long long)I.Nx * I.Ny, cidx = (long long)j * I.Nx + i;
    JacOut o;
    o.M = Pm.M;
    o.slot = perm2d(Pm, i, j);
    o.R0 = I.R[cidx];
    o.R1 = I.R[n + cidx];
    o.R2 = I.R[2 * n + cidx];
    o.rn = I.rn[cidx];
    o.alpha = I.alpha;
    o.eps = I.eps;
    if (rhs && col == 0) {
        rhs[o.slot] = (T)o.R0;
        rhs[o.M + o.slot] = (T)o.R1;
        rhs[2 * o.M + o.slot] = (T)o.R2;
    }
    const int pi = i + stencil_dx(21, b), pj = j + stencil_dy(21, b);
    if (pi < 0 || pi >= I.Nx || pj < 0 || pj >= I.Ny) {
        store_zero_column(J, o, b, m);
        return o.slot;
    }
    const GlobalStateT<SURF> st{I.U, I.zavg, I.Nx, I.Ny};
#pragma unroll 1
    for (int q = 0; q < kSlots; q++) {
        const V3 v = slot_state(I, st, q, i, j, pi, pj, m, I.eps);
#pragma unroll
        for (int c = 0; c < 3; c++) slots[(q * 3 + c) * kBorderNT + lane] = v.c[c];
    }
    double bx[4], by[4];
    load_slopes(I, i, j, bx, by);
    const SlotFS<SURF> fs{slots, lane};
    double h_own = 0.0;
    if constexpr (SURF) {
        const double x = st(0, i, j);
        h_own = (pi == i && pj == j && m == 0) ? x + I.eps : x;
    }
    const V3 Rp = assemble_residual(fs, I, bx, by, i, j, h_own);
    store_column(J, o, b, m, Rp, d);
    return o.slot;
}

// Jacobian of the border rows: one thread per (row, column of the stencil), each a full
// re-evaluation of the perturbed local residual from the state in global memory.  A row takes
// LPR lanes of a wavefront (32 for the 27 columns of J9, 64 for the 63 of J21), so the lanes of
// its three diagonal-block columns can hand their FP64 values to the row's first lane, which
// writes the inverse of the diagonal block.
template <typename T, int NB, bool SURF>
__global__ void __launch_bounds__(kBorderNT) k_jacobian2d_border(Inst2D I, Perm2D Pm, T *J, T *rhs, T *Dinv,
                                                                 long long nrows)
{
    constexpr int LPR = NB == 9 ? 32 : 64, LOG = NB == 9 ? 5 : 6;
    static_assert(kBorderNT % LPR == 0, "a workgroup holds whole rows");
    __shared__ double slots[kSlots * 3 * kBorderNT];
    const long long gid = blockIdx.x * (long long)kBorderNT + threadIdx.x;
    const long long r = gid >> LOG;
    const int col = (int)(gid & (LPR - 1)), b = col / 3, m = col - 3 * b;
    const bool active = r < nrows && col < 3 * NB;
    double d[3] = {0.0, 0.0, 0.0};
    long long slot = 0;
    if (active) slot = jacobian_border_column<T, SURF>(I, Pm, J, rhs, slots, threadIdx.x, r, col, d);
    if (!Dinv) return;   // uniform over the launch
    // the diagonal block's columns m = 0, 1, 2 sit in lanes 0, 1, 2 of the row's LPR
    const int base = threadIdx.x & ~(LPR - 1);
    double D[9];
#pragma unroll
    for (int mm = 0; mm < 3; mm++)
#pragma unroll
        for (int l = 0; l < 3; l++) D[l * 3 + mm] = __shfl(d[l], base + mm, 64);
    if (active && col == 0) store_dinv(Dinv, Pm.M, slot, D);
}

// ---- launchers ---------------------------------------------------------------------------

hipError_t launch_residual2d(const Inst2D &I, double *partial, hipStream_t s)
{
    dim3 grid((I.Nx + kTX - 1) / kTX, (I.Ny + kTY - 1) / kTY);
    if (I.recon == NMG_RECON_SURFACE) hipLaunchKernelGGL(k_residual2d<true>, grid, dim3(kTX, kTY), 0, s, I, partial);
    else hipLaunchKernelGGL(k_residual2d<false>, grid, dim3(kTX, kTY), 0, s, I, partial);
    return hipGetLastError();
}

int residual2d_tiles(int Nx, int Ny) { return ((Nx + kTX - 1) / kTX) * ((Ny + kTY - 1) / kTY); }

hipError_t launch_res2d_finalize(const double *partial, int ntiles, long long ncells, double *res,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(k_res2d_finalize, dim3(1), dim3(256), 0, s, partial, ntiles, ncells, res);
    return hipGetLastError();
}

template <typename T, int NB, bool SURF>
static hipError_t jacobian2d_t(const Inst2D &I, const Perm2D &P, T *J, T *rhs, T *Dinv, hipStream_t s)
{
    constexpr int LPR = NB == 9 ? 32 : 64;
    dim3 grid((I.Nx + kTX - 1) / kTX, (I.Ny + kTY - 1) / kTY);
    hipLaunchKernelGGL((k_jacobian2d<T, NB, SURF>), grid, dim3(kTX, kTY), 0, s, I, P, J, rhs, Dinv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long nb = border_rows2d(I.Nx, I.Ny);
    const long long blocks = (nb * LPR + kBorderNT - 1) / kBorderNT;
    hipLaunchKernelGGL((k_jacobian2d_border<T, NB, SURF>), dim3((unsigned)blocks), dim3(kBorderNT), 0, s, I, P, J,
                       rhs, Dinv, nb);
    return hipGetLastError();
}

template <typename T, bool SURF>
static hipError_t jacobian2d_nb(const Inst2D &I, const Perm2D &P, void *J, void *rhs, void *Dinv, int nb, hipStream_t s)
{
    if (nb == 21) return jacobian2d_t<T, 21, SURF>(I, P, (T *)J, (T *)rhs, (T *)Dinv, s);
    return jacobian2d_t<T, 9, SURF>(I, P, (T *)J, (T *)rhs, (T *)Dinv, s);
}

hipError_t launch_jacobian2d(const Inst2D &I, const Perm2D &P, void *J, void *rhs, void *Dinv, int prec,
                             hipStream_t s, int nb)
{
    if (nb != 9 && nb != 21) return hipErrorInvalidValue;
    const bool surf = I.recon == NMG_RECON_SURFACE;
    if (prec == NMG_FP32_MG)
        return surf ? jacobian2d_nb<float, true>(I, P, J, rhs, Dinv, nb, s) : jacobian2d_nb<float, false>(I, P, J, rhs, Dinv, nb, s);
    return surf ? jacobian2d_nb<double, true>(I, P, J, rhs, Dinv, nb, s) : jacobian2d_nb<double, false>(I, P, J, rhs, Dinv, nb, s);
}

}  // namespace nmg
