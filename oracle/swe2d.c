/*
 * CPU ORACLE -- test infrastructure only (two-dimensional part).
 *
 * Plain FP64 C implementation of the 2D NMGM of section 4 of the paper (Hu, Li, Wang, Wang):
 * the finite-volume residual of eq. (20) with characteristic WENO3 in each direction, Gauss
 * quadrature along faces and the tensor Gauss source, the finite-difference Jacobian on the
 * simplified cross stencil of eq. (21) (and the full 21-cell stencil), the coarse operators and
 * restriction of eq. (24), injection prolongation (eq. 25), the block SOR smoother of eq. (22)
 * in multicolour and in the four-direction sweeping order, a dense direct solve on the coarsest
 * grid, Algorithm 2 and Algorithm 1.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it; it shares nothing with the GPU library.
 *
 * Conventions.  Cell (i, j), i = 0..Nx-1 (x), j = 0..Ny-1 (y).  U = (h, hu, hv) stored
 * component-major U[(c*Ny + j)*Nx + i].  Geometry: b_x and b_y at the tensor Gauss points of
 * each cell, [(j*Nx + i)*4 + 2*beta + gamma] with beta the y point and gamma the x point (0 the
 * lower/left point x_i - dx/(2 sqrt 3)).
 *
 * Readings (listed in the design notes):
 *  Q1  The face values U^-+_{i+1/2,j} come from 1D WENO in x of 2D cell averages, hence are
 *      averages along the face; the quadratic in y through three of them (the A.1 form)
 *      evaluated at the Gauss points is V_j +- (V_{j+1} - V_{j-1}) / (4 sqrt 3) (its curvature
 *      term vanishes there): P = V_j + t (V_{j+1} - V_{j-1}) / 2, t = -+1/(2 sqrt 3).
 *  Q2  Characteristic decomposition: eigenvectors of the face-normal flux Jacobian (section 2)
 *      at the arithmetic mean of the two cells sharing the face; the three stencil cells are
 *      projected on the left eigenvectors, each field gets scalar WENO3 (third-order weights as
 *      in 1D), and the result is mapped back with the right eigenvectors.
 *  Q3  LLF flux with the local speed max(|u_n| + sqrt(g h)) over both states at each Gauss point.
 *  Q4  Ghost cells: y sides first, then x sides (corners = x rule applied to the y ghost);
 *      EXTRAP copies the boundary cell, WALL mirrors (ghost k = cell k-1 from the wall) with the
 *      normal momentum negated, STATE gives (h, h u, h v), DISCHARGE copies h and hv and sets the
 *      normal discharge, DEPTH sets h and copies the momenta.  The bottom side may be EXTRAP for
 *      cell centres x < wall_x and WALL beyond.
 *  S1  Surface variant (recon = 1), so that still water is steady on any bottom: the WENO
 *      reconstructions act on (eta, hu, hv) with eta = h + zbar (zbar the cell average of b; the
 *      characteristic basis still at the mean of the two cells' (h, hu, hv)); the depth at a
 *      face Gauss point is eta there minus b at that point; a ghost that copies the depth of a
 *      grid cell copies its surface instead (h_g = h_src + zbar_src - zbar_g); the source of
 *      each Gauss line is the exactly equal split form
 *        -g [ int (eta_h - eta_ij) b_x + eta_ij (b_+ - b_-) - (b_+^2 - b_-^2) / 2 ]
 *      (eta_h the cubic through the four face values of eta on that line, the integral by the
 *      same two-point Gauss rule, b_-+ at the cell's faces on that line), summed over the two
 *      Gauss lines with weight (cell width across) / 2.  With b = 0 it is the paper's scheme.
 *  Q5  Multicolour smoothing: colour (i + j) mod C, C = 3 on the cross stencil (offsets up to 2),
 *      2 on five-point levels; on the full 21-cell stencil, whose diagonal neighbours (1, -1)
 *      share (i + j) mod 3, nine colours (i mod 3) + 3 (j mod 3).  With these colourings no
 *      two cells of one colour are coupled, so a colour sweep is a simultaneous block-Jacobi
 *      update of its cells.  One smoothing iteration = four colour sweeps (forward, backward,
 *      forward, backward), the analogue of the four directional sweeps D1-D4.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_BC_DISCHARGE 0
#define OR_BC_DEPTH 1
#define OR_BC_EXTRAP 2
#define OR_BC_WALL 3
#define OR_BC_STATE 4

typedef struct {
    int Nx, Ny;
    double dx, dy, g, x0, y0;
    const double *bx_gp;   /* [Ny][Nx][2][2] */
    const double *by_gp;
    int bc_kind[4];        /* left, right, bottom, top */
    double bc_q[4], bc_h[4], bc_u[4], bc_v[4];
    double wall_x;         /* bottom: EXTRAP for x < wall_x, WALL beyond (when wall_x > x0) */
    int recon;             /* 0: reconstruct (h, hu, hv) (the paper); 1: the surface variant S1 */
    const double *zavg;    /* recon 1: cell averages of b over cells -2..Nx+1 x -2..Ny+1, [Ny+4][Nx+4] */
    const double *zfx;     /* recon 1: b at the Gauss points of the x faces, [Ny][Nx+1][2] */
    const double *zfy;     /* recon 1: b at the Gauss points of the y faces, [Ny+1][Nx][2] */
} or2d_prob;

typedef struct {
    double alpha, tau, eps, omega, tol;
    int nu1, nu2, nu3, n_max;
    int levels;
    int stencil;   /* 9: simplified J9; 21: full J21 */
    int smoother;  /* 0 multicolour, 1 four-direction sweeps */
} or2d_params;

static const double ZETA2 = 1e-6;

#define UIDX(p, c, i, j) (((c) * (p)->Ny + (j)) * (p)->Nx + (i))
#define ZAVG(p, i, j) ((p)->zavg[((j) + 2) * ((p)->Nx + 4) + (i) + 2])

/* ---- ghost cells (reading Q4) ------------------------------------------------------------ */

static int bottom_kind(const or2d_prob *p, int i)
{
    if (p->bc_kind[2] == OR_BC_WALL && p->wall_x > p->x0) {
        double xc = p->x0 + (i + 0.5) * p->dx;
        return xc < p->wall_x ? OR_BC_EXTRAP : OR_BC_WALL;
    }
    return p->bc_kind[2];
}

/* Value of cell (i, j) of the state U, for any i, j within two cells of the grid. */
void or2d_cell(const or2d_prob *p, const double *U, int i, int j, double out[3])
{
    int ii = i, jj = j, flip_u = 0, flip_v = 0, state = -1, set_h = -1, set_q = -1;
    if (j < 0 || j >= p->Ny) {
        int side = j < 0 ? 2 : 3;
        int kind = side == 2 ? bottom_kind(p, i) : p->bc_kind[3];
        int b = j < 0 ? 0 : p->Ny - 1;
        int m = j < 0 ? -1 - j : 2 * p->Ny - 1 - j;
        jj = b;
        if (kind == OR_BC_WALL) { jj = m; flip_v = 1; }
        else if (kind == OR_BC_STATE) state = side;
        else if (kind == OR_BC_DISCHARGE) set_q = side;
        else if (kind == OR_BC_DEPTH) set_h = side;
    }
    if (i < 0 || i >= p->Nx) {
        int side = i < 0 ? 0 : 1;
        int kind = p->bc_kind[side];
        int b = i < 0 ? 0 : p->Nx - 1;
        int m = i < 0 ? -1 - i : 2 * p->Nx - 1 - i;
        ii = b;
        if (kind == OR_BC_WALL) { ii = m; flip_u = 1; }
        else if (kind == OR_BC_STATE) state = side;
        else if (kind == OR_BC_DISCHARGE) set_q = side;
        else if (kind == OR_BC_DEPTH) set_h = side;
    }
    if (state >= 0) {
        out[0] = p->bc_h[state];
        out[1] = p->bc_h[state] * p->bc_u[state];
        out[2] = p->bc_h[state] * p->bc_v[state];
        return;
    }
    out[0] = U[UIDX(p, 0, ii, jj)];
    out[1] = U[UIDX(p, 1, ii, jj)];
    out[2] = U[UIDX(p, 2, ii, jj)];
    if (flip_u) out[1] = -out[1];
    if (flip_v) out[2] = -out[2];
    if (p->recon == 1 && (ii != i || jj != j)) out[0] = out[0] + ZAVG(p, ii, jj) - ZAVG(p, i, j);   /* S1 */
    if (set_h >= 0) out[0] = p->bc_h[set_h];
    if (set_q >= 0) {
        if (set_q < 2) out[1] = p->bc_q[set_q];
        else out[2] = p->bc_q[set_q];
    }
}

/* ---- characteristic WENO3 (readings Q2, eq. 7-8 per field) --------------------------------- */

static double weno_p(double um, double u0, double up)
{
    double c0 = 1.5 * u0 - 0.5 * up;
    double c1 = 0.5 * um + 0.5 * u0;
    double b0 = (up - u0) * (up - u0);
    double b1 = (u0 - um) * (u0 - um);
    double a0 = (1.0 / 3.0) / ((ZETA2 + b0) * (ZETA2 + b0));
    double a1 = (2.0 / 3.0) / ((ZETA2 + b1) * (ZETA2 + b1));
    double w0 = a0 / (a0 + a1);
    double w1 = a1 / (a0 + a1);
    return w0 * c0 + w1 * c1;
}

static double weno_m(double um, double u0, double up)
{
    double c0 = 0.5 * u0 + 0.5 * up;
    double c1 = -0.5 * um + 1.5 * u0;
    double b0 = (up - u0) * (up - u0);
    double b1 = (u0 - um) * (u0 - um);
    double a0 = (2.0 / 3.0) / ((ZETA2 + b0) * (ZETA2 + b0));
    double a1 = (1.0 / 3.0) / ((ZETA2 + b1) * (ZETA2 + b1));
    double w0 = a0 / (a0 + a1);
    double w1 = a1 / (a0 + a1);
    return w0 * c0 + w1 * c1;
}

/* Left (L) and right (R) eigenvectors of the flux Jacobian in direction dir (0: x, 1: y) at
 * the state Us: eigenvalues u_n - c, u_n, u_n + c (section 2). */
void or2d_eigen(const double Us[3], int dir, double g, double L[3][3], double R[3][3])
{
    double h = Us[0];
    double u = Us[1] / h;
    double v = Us[2] / h;
    double c = sqrt(g * h);
    double un = dir == 0 ? u : v;
    double i2c = 1.0 / (2.0 * c);
    /* L rows */
    if (dir == 0) {
        L[0][0] = (un + c) * i2c; L[0][1] = -i2c; L[0][2] = 0.0;
        L[1][0] = -v;             L[1][1] = 0.0;  L[1][2] = 1.0;
        L[2][0] = -(un - c) * i2c; L[2][1] = i2c; L[2][2] = 0.0;
        R[0][0] = 1.0;    R[0][1] = 0.0; R[0][2] = 1.0;
        R[1][0] = un - c; R[1][1] = 0.0; R[1][2] = un + c;
        R[2][0] = v;      R[2][1] = 1.0; R[2][2] = v;
    } else {
        L[0][0] = (un + c) * i2c; L[0][1] = 0.0; L[0][2] = -i2c;
        L[1][0] = -u;             L[1][1] = 1.0; L[1][2] = 0.0;
        L[2][0] = -(un - c) * i2c; L[2][1] = 0.0; L[2][2] = i2c;
        R[0][0] = 1.0;    R[0][1] = 0.0; R[0][2] = 1.0;
        R[1][0] = u;      R[1][1] = 1.0; R[1][2] = u;
        R[2][0] = un - c; R[2][1] = 0.0; R[2][2] = un + c;
    }
}

/* State at the face between cells a and a+1 of a line (dir 0: row k, cells (a, k); dir 1:
 * column k, cells (k, a)), reconstructed from cell a (which = 0, the minus state) or from cell
 * a+1 (which = 1, the plus state). */
void or2d_face_state(const or2d_prob *p, const double *U, int dir, int k, int a, int which, double out[3])
{
    double Ua[3], Ub[3], S[3][3], Us[3], L[3][3], R[3][3];
#define CELL(t, o) (dir == 0 ? or2d_cell(p, U, (t), k, (o)) : or2d_cell(p, U, k, (t), (o)))
    CELL(a, Ua);
    CELL(a + 1, Ub);
    for (int c = 0; c < 3; c++) Us[c] = 0.5 * (Ua[c] + Ub[c]);
    or2d_eigen(Us, dir, p->g, L, R);
    int m = which ? a + 1 : a;
    CELL(m - 1, S[0]);
    CELL(m, S[1]);
    CELL(m + 1, S[2]);
#undef CELL
    if (p->recon == 1)   /* S1: reconstruct the surface */
        for (int s = 0; s < 3; s++)
            S[s][0] = S[s][0] + (dir == 0 ? ZAVG(p, m - 1 + s, k) : ZAVG(p, k, m - 1 + s));
    double W[3][3], w[3];
    for (int s = 0; s < 3; s++)
        for (int f = 0; f < 3; f++)
            W[s][f] = L[f][0] * S[s][0] + L[f][1] * S[s][1] + L[f][2] * S[s][2];
    for (int f = 0; f < 3; f++)
        w[f] = which ? weno_p(W[0][f], W[1][f], W[2][f]) : weno_m(W[0][f], W[1][f], W[2][f]);
    for (int c = 0; c < 3; c++)
        out[c] = R[c][0] * w[0] + R[c][1] * w[1] + R[c][2] * w[2];
}

/* ---- physical fluxes and LLF (reading Q3) -------------------------------------------------- */

void or2d_flux(const double U[3], int dir, double g, double F[3])
{
    double h = U[0];
    double u = U[1] / h;
    double v = U[2] / h;
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

void or2d_llf(const double UL[3], const double UR[3], int dir, double g, double F[3])
{
    double FL[3], FR[3];
    or2d_flux(UL, dir, g, FL);
    or2d_flux(UR, dir, g, FR);
    double unL = UL[1 + dir] / UL[0], unR = UR[1 + dir] / UR[0];
    double sL = fabs(unL) + sqrt(g * UL[0]);
    double sR = fabs(unR) + sqrt(g * UR[0]);
    double a = sL > sR ? sL : sR;
    for (int c = 0; c < 3; c++)
        F[c] = 0.5 * (FL[c] + FR[c] - a * (UR[c] - UL[c]));
}

/* ---- local residual, eq. (20) -------------------------------------------------------------- */

static void gauss_line(const double Vm[3], const double V0[3], const double Vp[3], double P[2][3])
{
    /* reading Q1: P_beta = V0 + t_beta (Vp - Vm) / 2, t = -+1/(2 sqrt 3) */
    double t0 = -1.0 / (2.0 * sqrt(3.0)), t1 = 1.0 / (2.0 * sqrt(3.0));
    for (int c = 0; c < 3; c++) {
        double slope = (Vp[c] - Vm[c]) * 0.5;
        P[0][c] = V0[c] + t0 * slope;
        P[1][c] = V0[c] + t1 * slope;
    }
}

/* Edge-averaged flux through the face between cells (a, j) and (a+1, j) (dir 0), or between
 * (i, a) and (i, a+1) (dir 1): two-point Gauss rule along the face of the LLF flux of the
 * states interpolated from the neighbouring lines.  Also returns the depth of both states at
 * the two Gauss points (for the source). */
void or2d_face_flux(const or2d_prob *p, const double *U, int dir, int line, int a, double F[3],
                    double hm[2], double hp[2])
{
    double Vm[3][3], Vp[3][3], Pm[2][3], Pp[2][3];
    for (int s = 0; s < 3; s++) {
        or2d_face_state(p, U, dir, line - 1 + s, a, 0, Vm[s]);
        or2d_face_state(p, U, dir, line - 1 + s, a, 1, Vp[s]);
    }
    gauss_line(Vm[0], Vm[1], Vm[2], Pm);
    gauss_line(Vp[0], Vp[1], Vp[2], Pp);
    if (hm) { hm[0] = Pm[0][0]; hm[1] = Pm[1][0]; }
    if (hp) { hp[0] = Pp[0][0]; hp[1] = Pp[1][0]; }
    if (p->recon == 1)   /* S1: the depth at each Gauss point is the surface minus b there */
        for (int q = 0; q < 2; q++) {
            double b = dir == 0 ? p->zfx[(line * (p->Nx + 1) + a + 1) * 2 + q]
                                : p->zfy[((a + 1) * p->Nx + line) * 2 + q];
            Pm[q][0] = Pm[q][0] - b;
            Pp[q][0] = Pp[q][0] - b;
        }
    double F0[3], F1[3];
    or2d_llf(Pm[0], Pp[0], dir, p->g, F0);
    or2d_llf(Pm[1], Pp[1], dir, p->g, F1);
    for (int c = 0; c < 3; c++) F[c] = 0.5 * (F0[c] + F1[c]);
}

/* depth of one face state at the two Gauss points along the face */
static void face_depth(const or2d_prob *p, const double *U, int dir, int line, int a, int which,
                       double hg[2])
{
    double V[3][3], P[2][3];
    for (int s = 0; s < 3; s++) or2d_face_state(p, U, dir, line - 1 + s, a, which, V[s]);
    gauss_line(V[0], V[1], V[2], P);
    hg[0] = P[0][0];
    hg[1] = P[1][0];
}

void or2d_cubic_weights(double Wt[2][4])
{
    const double nodes[4] = {-1.5, -0.5, 0.5, 1.5};
    double tg[2];
    tg[0] = -1.0 / (2.0 * sqrt(3.0));
    tg[1] = 1.0 / (2.0 * sqrt(3.0));
    for (int q = 0; q < 2; q++)
        for (int k = 0; k < 4; k++) {
            double w = 1.0;
            for (int m = 0; m < 4; m++)
                if (m != k) w *= (tg[q] - nodes[m]) / (nodes[k] - nodes[m]);
            Wt[q][k] = w;
        }
}

void or2d_local_residual(const or2d_prob *p, const double *U, int i, int j, double R[3])
{
    double fxm[3], fxp[3], fym[3], fyp[3];
    /* inner interface depths along the Gauss lines: [node][gauss point] */
    double hx[4][2], hy[4][2];
    or2d_face_flux(p, U, 0, j, i - 1, fxm, NULL, hx[1]);   /* x_{i-1/2}: plus state, from cell i */
    or2d_face_flux(p, U, 0, j, i, fxp, hx[2], NULL);       /* x_{i+1/2}: minus state, from cell i */
    or2d_face_flux(p, U, 1, i, j - 1, fym, NULL, hy[1]);
    or2d_face_flux(p, U, 1, i, j, fyp, hy[2], NULL);
    face_depth(p, U, 0, j, i - 2, 1, hx[0]);                /* x_{i-3/2}: plus state, cell i-1 */
    face_depth(p, U, 0, j, i + 1, 0, hx[3]);                /* x_{i+3/2}: minus state, cell i+1 */
    face_depth(p, U, 1, i, j - 2, 1, hy[0]);
    face_depth(p, U, 1, i, j + 1, 0, hy[3]);

    double Wt[2][4];
    or2d_cubic_weights(Wt);
    const double *bx = &p->bx_gp[(j * p->Nx + i) * 4];
    const double *by = &p->by_gp[(j * p->Nx + i) * 4];
    /* S2: cubic in x along each y Gauss line beta, at the x Gauss points gamma */
    double s2 = 0.0;
    for (int be = 0; be < 2; be++)
        for (int ga = 0; ga < 2; ga++) {
            double h = Wt[ga][0] * hx[0][be] + Wt[ga][1] * hx[1][be] + Wt[ga][2] * hx[2][be] + Wt[ga][3] * hx[3][be];
            s2 = s2 + p->g * h * bx[2 * be + ga];
        }
    /* S3: cubic in y along each x Gauss line gamma, at the y Gauss points beta */
    double s3 = 0.0;
    for (int ga = 0; ga < 2; ga++)
        for (int be = 0; be < 2; be++) {
            double h = Wt[be][0] * hy[0][ga] + Wt[be][1] * hy[1][ga] + Wt[be][2] * hy[2][ga] + Wt[be][3] * hy[3][ga];
            s3 = s3 + p->g * h * by[2 * be + ga];
        }
    double S2 = -(p->dx * p->dy / 4.0) * s2;
    double S3 = -(p->dx * p->dy / 4.0) * s3;
    if (p->recon == 1) {
        /* S1: hx, hy hold the surface; the split form of the source */
        double eta = U[UIDX(p, 0, i, j)] + ZAVG(p, i, j);
        s2 = 0.0;
        for (int be = 0; be < 2; be++)
            for (int ga = 0; ga < 2; ga++) {
                double e = Wt[ga][0] * hx[0][be] + Wt[ga][1] * hx[1][be] + Wt[ga][2] * hx[2][be] + Wt[ga][3] * hx[3][be];
                s2 = s2 + p->g * (e - eta) * bx[2 * be + ga];
            }
        double e2 = 0.0;
        for (int be = 0; be < 2; be++) {
            double bm = p->zfx[(j * (p->Nx + 1) + i) * 2 + be], bp = p->zfx[(j * (p->Nx + 1) + i + 1) * 2 + be];
            e2 = e2 + p->g * (eta * (bp - bm) - (bp * bp - bm * bm) / 2.0);
        }
        s3 = 0.0;
        for (int ga = 0; ga < 2; ga++)
            for (int be = 0; be < 2; be++) {
                double e = Wt[be][0] * hy[0][ga] + Wt[be][1] * hy[1][ga] + Wt[be][2] * hy[2][ga] + Wt[be][3] * hy[3][ga];
                s3 = s3 + p->g * (e - eta) * by[2 * be + ga];
            }
        double e3 = 0.0;
        for (int ga = 0; ga < 2; ga++) {
            double bm = p->zfy[(j * p->Nx + i) * 2 + ga], bp = p->zfy[((j + 1) * p->Nx + i) * 2 + ga];
            e3 = e3 + p->g * (eta * (bp - bm) - (bp * bp - bm * bm) / 2.0);
        }
        S2 = -(p->dx * p->dy / 4.0) * s2 - (p->dy / 2.0) * e2;
        S3 = -(p->dx * p->dy / 4.0) * s3 - (p->dx / 2.0) * e3;
    }
    R[0] = (fxp[0] - fxm[0]) / p->dx + (fyp[0] - fym[0]) / p->dy;
    R[1] = (fxp[1] - fxm[1]) / p->dx + (fyp[1] - fym[1]) / p->dy - S2 / (p->dx * p->dy);
    R[2] = (fxp[2] - fxm[2]) / p->dx + (fyp[2] - fym[2]) / p->dy - S3 / (p->dx * p->dy);
}

double or2d_residual(const or2d_prob *p, const double *U, double *R, double *rn)
{
    int Nx = p->Nx, Ny = p->Ny;
    double sum = 0.0;
    for (int j = 0; j < Ny; j++)
        for (int i = 0; i < Nx; i++) {
            double r[3];
            or2d_local_residual(p, U, i, j, r);
            for (int c = 0; c < 3; c++) R[UIDX(p, c, i, j)] = r[c];
            double n1 = fabs(r[0]) + fabs(r[1]) + fabs(r[2]);
            if (rn) rn[j * Nx + i] = n1;
            sum += n1;
        }
    return sum / (Nx * Ny);
}

/* ---- finite-difference Jacobian (eq. 12, 13, 21) --------------------------------------------- */

/* stencil offsets: the simplified cross of eq. (21) (centre first), and the full 21 cells */
static const int OFF9[9][2] = {{0, 0}, {-2, 0}, {-1, 0}, {1, 0}, {2, 0}, {0, -2}, {0, -1}, {0, 1}, {0, 2}};

int or2d_stencil(int which, int off[21][2])
{
    if (which == 9) {
        for (int k = 0; k < 9; k++) { off[k][0] = OFF9[k][0]; off[k][1] = OFF9[k][1]; }
        return 9;
    }
    int n = 0;
    for (int k = 0; k < 9; k++) { off[n][0] = OFF9[k][0]; off[n][1] = OFF9[k][1]; n++; }
    for (int dj = -1; dj <= 1; dj += 2)
        for (int di = -2; di <= 2; di++) if (di != 0) { off[n][0] = di; off[n][1] = dj; n++; }
    for (int di = -1; di <= 1; di += 2)
        for (int dj = -2; dj <= 2; dj += 2) if (dj != 0) { off[n][0] = di; off[n][1] = dj; n++; }
    return n;
}

/* J blocks [Ny][Nx][nb][3][3] for the row cells in [j0, j1): column (p, q, m) perturbs U_pq^m
 * by eps in the state vector (ghosts follow), the forward difference of R_ij. */
void or2d_jacobian_rows(const or2d_prob *p, const double *U, const double *R, const double *rn,
                        double eps, double alpha, int which, int j0, int j1, double *J)
{
    int off[21][2];
    int nb = or2d_stencil(which, off);
    int Nx = p->Nx, Ny = p->Ny;
    double *Up = malloc(sizeof(double) * 3 * Nx * Ny);
    memcpy(Up, U, sizeof(double) * 3 * Nx * Ny);
    for (int j = j0; j < j1; j++)
        for (int i = 0; i < Nx; i++) {
            double *Jc = &J[(size_t)((j * Nx + i) * nb) * 9];
            for (int b = 0; b < nb; b++) {
                int pi = i + off[b][0], pj = j + off[b][1];
                for (int m = 0; m < 3; m++) {
                    double col[3] = {0.0, 0.0, 0.0};
                    if (pi >= 0 && pi < Nx && pj >= 0 && pj < Ny) {
                        double saved = Up[UIDX(p, m, pi, pj)];
                        Up[UIDX(p, m, pi, pj)] = saved + eps;
                        double Rp[3];
                        or2d_local_residual(p, Up, i, j, Rp);
                        Up[UIDX(p, m, pi, pj)] = saved;
                        for (int l = 0; l < 3; l++) col[l] = (Rp[l] - R[UIDX(p, l, i, j)]) / eps;
                    }
                    for (int l = 0; l < 3; l++) Jc[b * 9 + l * 3 + m] = col[l];
                }
            }
            for (int l = 0; l < 3; l++) Jc[l * 3 + l] += alpha * rn[j * Nx + i];
        }
    free(Up);
}

void or2d_jacobian(const or2d_prob *p, const double *U, const double *R, const double *rn,
                   double eps, double alpha, int which, double *J)
{
    int rows = p->Ny;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < rows; j++)
        or2d_jacobian_rows(p, U, R, rn, eps, alpha, which, j, j + 1, J);
}

/* ---- multigrid (section 4.2) ----------------------------------------------------------------- */

typedef struct {
    int nlev;
    int nx[32], ny[32], nb[32];
    int off[32][21][2];
    double *J[32], *Dinv[32], *rhs[32], *dU[32];   /* rhs, dU: [ny][nx][3] */
} or2d_mg;

static const int OFF5[5][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}};

static int find_off(const or2d_mg *mg, int l, int di, int dj)
{
    for (int b = 0; b < mg->nb[l]; b++)
        if (mg->off[l][b][0] == di && mg->off[l][b][1] == dj) return b;
    return -1;
}

static void inv3(const double A[9], double B[9])
{
    double c00 = A[4] * A[8] - A[5] * A[7];
    double c01 = A[5] * A[6] - A[3] * A[8];
    double c02 = A[3] * A[7] - A[4] * A[6];
    double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
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

or2d_mg *or2d_mg_create(int nx, int ny, int levels, int which)
{
    or2d_mg *mg = calloc(1, sizeof(or2d_mg));
    mg->nlev = levels;
    for (int l = 0; l < levels; l++) {
        mg->nx[l] = nx >> l;
        mg->ny[l] = ny >> l;
        if (l == 0) {
            mg->nb[l] = or2d_stencil(which, mg->off[l]);
        } else {
            mg->nb[l] = 5;
            for (int b = 0; b < 5; b++) { mg->off[l][b][0] = OFF5[b][0]; mg->off[l][b][1] = OFF5[b][1]; }
        }
        size_t n = (size_t)mg->nx[l] * mg->ny[l];
        mg->J[l] = calloc(n * mg->nb[l] * 9, sizeof(double));
        mg->Dinv[l] = calloc(n * 9, sizeof(double));
        mg->rhs[l] = calloc(n * 3, sizeof(double));
        mg->dU[l] = calloc(n * 3, sizeof(double));
    }
    return mg;
}

void or2d_mg_free(or2d_mg *mg)
{
    for (int l = 0; l < mg->nlev; l++) { free(mg->J[l]); free(mg->Dinv[l]); free(mg->rhs[l]); free(mg->dU[l]); }
    free(mg);
}

/* eq. (24), operator part: J^{IJ}_{PQ,l} = sum over the 2x2 children (row) and the 2x2 children
 * of (P, Q) (column) of the fine blocks; coarse offsets are the five-point set. */
void or2d_coarsen_level(or2d_mg *mg, int l)
{
    int nxf = mg->nx[l - 1], nyf = mg->ny[l - 1], nbf = mg->nb[l - 1];
    int nxc = mg->nx[l], nyc = mg->ny[l];
    double *Jc = mg->J[l];
    memset(Jc, 0, sizeof(double) * (size_t)nxc * nyc * 5 * 9);
    for (int J_ = 0; J_ < nyc; J_++)
        for (int I = 0; I < nxc; I++)
            for (int bc = 0; bc < 5; bc++) {
                int P = I + OFF5[bc][0], Q = J_ + OFF5[bc][1];
                if (P < 0 || P >= nxc || Q < 0 || Q >= nyc) continue;
                double *blk = &Jc[((J_ * nxc + I) * 5 + bc) * 9];
                for (int fj = 2 * J_; fj <= 2 * J_ + 1; fj++)
                    for (int fi = 2 * I; fi <= 2 * I + 1; fi++)
                        for (int cj = 2 * Q; cj <= 2 * Q + 1; cj++)
                            for (int ci = 2 * P; ci <= 2 * P + 1; ci++) {
                                int b = find_off(mg, l - 1, ci - fi, cj - fj);
                                if (b < 0) continue;
                                const double *src = &mg->J[l - 1][((fj * nxf + fi) * nbf + b) * 9];
                                for (int e = 0; e < 9; e++) blk[e] = blk[e] + src[e];
                            }
            }
    (void)nyf;
}

void or2d_mg_setup(or2d_mg *mg, const double *Jfine)
{
    size_t n0 = (size_t)mg->nx[0] * mg->ny[0];
    memcpy(mg->J[0], Jfine, sizeof(double) * n0 * mg->nb[0] * 9);
    for (int l = 1; l < mg->nlev; l++) or2d_coarsen_level(mg, l);
    for (int l = 0; l < mg->nlev; l++) {
        size_t n = (size_t)mg->nx[l] * mg->ny[l];
        for (size_t k = 0; k < n; k++) inv3(&mg->J[l][(k * mg->nb[l]) * 9], &mg->Dinv[l][k * 9]);
    }
}

double *or2d_mg_level_J(or2d_mg *mg, int l) { return mg->J[l]; }
double *or2d_mg_level_rhs(or2d_mg *mg, int l) { return mg->rhs[l]; }
double *or2d_mg_level_dU(or2d_mg *mg, int l) { return mg->dU[l]; }

/* eq. (22): one block SOR update of cell (i, j) */
static void sor2(or2d_mg *mg, int l, int i, int j, double omega)
{
    int nx = mg->nx[l], ny = mg->ny[l], nb = mg->nb[l];
    double *dU = mg->dU[l];
    double r[3];
    for (int c = 0; c < 3; c++) r[c] = mg->rhs[l][(j * nx + i) * 3 + c];
    for (int b = 1; b < nb; b++) {
        int pi = i + mg->off[l][b][0], pj = j + mg->off[l][b][1];
        if (pi < 0 || pi >= nx || pj < 0 || pj >= ny) continue;
        const double *blk = &mg->J[l][((j * nx + i) * nb + b) * 9];
        const double *x = &dU[(pj * nx + pi) * 3];
        for (int c = 0; c < 3; c++) r[c] = r[c] + (blk[c * 3 + 0] * x[0] + blk[c * 3 + 1] * x[1] + blk[c * 3 + 2] * x[2]);
    }
    const double *D = &mg->Dinv[l][(j * nx + i) * 9];
    double t[3];
    for (int c = 0; c < 3; c++) t[c] = D[c * 3 + 0] * r[0] + D[c * 3 + 1] * r[1] + D[c * 3 + 2] * r[2];
    for (int c = 0; c < 3; c++) dU[(j * nx + i) * 3 + c] = (1.0 - omega) * dU[(j * nx + i) * 3 + c] - omega * t[c];
}

/* colour of cell (i, j) among C (reading Q5) */
static int colour_of(int i, int j, int C)
{
    return C == 9 ? i % 3 + 3 * (j % 3) : (i + j) % C;
}

/* one smoothing iteration (reading Q5; smoother 1: the sweeps D1-D4 of section 4.2) */
void or2d_smooth(or2d_mg *mg, int l, double omega, int smoother)
{
    int nx = mg->nx[l], ny = mg->ny[l];
    if (smoother == 1) {
        for (int i = 0; i < nx; i++) for (int j = 0; j < ny; j++) sor2(mg, l, i, j, omega);            /* D1 */
        for (int i = nx - 1; i >= 0; i--) for (int j = 0; j < ny; j++) sor2(mg, l, i, j, omega);       /* D2 */
        for (int i = nx - 1; i >= 0; i--) for (int j = ny - 1; j >= 0; j--) sor2(mg, l, i, j, omega);  /* D3 */
        for (int i = 0; i < nx; i++) for (int j = ny - 1; j >= 0; j--) sor2(mg, l, i, j, omega);       /* D4 */
        return;
    }
    int C = mg->nb[l] == 5 ? 2 : (mg->nb[l] == 21 ? 9 : 3);
    for (int rep = 0; rep < 2; rep++) {
        for (int c = 0; c < C; c++)
            for (int j = 0; j < ny; j++) for (int i = 0; i < nx; i++) if (colour_of(i, j, C) == c) sor2(mg, l, i, j, omega);
        for (int c = C - 1; c >= 0; c--)
            for (int j = 0; j < ny; j++) for (int i = 0; i < nx; i++) if (colour_of(i, j, C) == c) sor2(mg, l, i, j, omega);
    }
}

void or2d_coarse_solve(or2d_mg *mg, int l)
{
    int nx = mg->nx[l], ny = mg->ny[l], nb = mg->nb[l], M = 3 * nx * ny;
    double *A = calloc((size_t)M * M, sizeof(double));
    double *x = calloc(M, sizeof(double));
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++)
            for (int b = 0; b < nb; b++) {
                int pi = i + mg->off[l][b][0], pj = j + mg->off[l][b][1];
                if (pi < 0 || pi >= nx || pj < 0 || pj >= ny) continue;
                const double *blk = &mg->J[l][((j * nx + i) * nb + b) * 9];
                for (int r = 0; r < 3; r++)
                    for (int c = 0; c < 3; c++)
                        A[(size_t)((j * nx + i) * 3 + r) * M + (pj * nx + pi) * 3 + c] = blk[r * 3 + c];
            }
    for (int r = 0; r < M; r++) x[r] = -mg->rhs[l][r];
    for (int k = 0; k < M; k++) {
        int piv = k;
        for (int r = k + 1; r < M; r++)
            if (fabs(A[(size_t)r * M + k]) > fabs(A[(size_t)piv * M + k])) piv = r;
        if (piv != k) {
            for (int c = 0; c < M; c++) { double t = A[(size_t)k * M + c]; A[(size_t)k * M + c] = A[(size_t)piv * M + c]; A[(size_t)piv * M + c] = t; }
            double t = x[k]; x[k] = x[piv]; x[piv] = t;
        }
        for (int r = k + 1; r < M; r++) {
            double f = A[(size_t)r * M + k] / A[(size_t)k * M + k];
            if (f == 0.0) continue;
            for (int c = k; c < M; c++) A[(size_t)r * M + c] -= f * A[(size_t)k * M + c];
            x[r] -= f * x[k];
        }
    }
    for (int k = M - 1; k >= 0; k--) {
        double s = x[k];
        for (int c = k + 1; c < M; c++) s -= A[(size_t)k * M + c] * x[c];
        x[k] = s / A[(size_t)k * M + k];
    }
    memcpy(mg->dU[l], x, sizeof(double) * M);
    free(A);
    free(x);
}

/* eq. (24), right-hand side */
void or2d_restrict(or2d_mg *mg, int l)
{
    int nx = mg->nx[l], ny = mg->ny[l], nb = mg->nb[l], nxc = mg->nx[l + 1], nyc = mg->ny[l + 1];
    for (int J_ = 0; J_ < nyc; J_++)
        for (int I = 0; I < nxc; I++) {
            double s[3] = {0.0, 0.0, 0.0};
            for (int fj = 2 * J_; fj <= 2 * J_ + 1; fj++)
                for (int fi = 2 * I; fi <= 2 * I + 1; fi++) {
                    double a[3];
                    for (int c = 0; c < 3; c++) a[c] = mg->rhs[l][(fj * nx + fi) * 3 + c];
                    for (int b = 0; b < nb; b++) {
                        int pi = fi + mg->off[l][b][0], pj = fj + mg->off[l][b][1];
                        if (pi < 0 || pi >= nx || pj < 0 || pj >= ny) continue;
                        const double *blk = &mg->J[l][((fj * nx + fi) * nb + b) * 9];
                        const double *x = &mg->dU[l][(pj * nx + pi) * 3];
                        for (int c = 0; c < 3; c++) a[c] = a[c] + (blk[c * 3 + 0] * x[0] + blk[c * 3 + 1] * x[1] + blk[c * 3 + 2] * x[2]);
                    }
                    for (int c = 0; c < 3; c++) s[c] = s[c] + a[c];
                }
            for (int c = 0; c < 3; c++) mg->rhs[l + 1][(J_ * nxc + I) * 3 + c] = s[c];
        }
}

/* eq. (25) */
void or2d_prolong(or2d_mg *mg, int l)
{
    int nx = mg->nx[l], nxc = mg->nx[l + 1], nyc = mg->ny[l + 1];
    for (int J_ = 0; J_ < nyc; J_++)
        for (int I = 0; I < nxc; I++)
            for (int fj = 2 * J_; fj <= 2 * J_ + 1; fj++)
                for (int fi = 2 * I; fi <= 2 * I + 1; fi++)
                    for (int c = 0; c < 3; c++)
                        mg->dU[l][(fj * nx + fi) * 3 + c] += mg->dU[l + 1][(J_ * nxc + I) * 3 + c];
}

void or2d_vcycle(or2d_mg *mg, int l, double omega, int nu1, int nu2, int smoother)
{
    if (l == mg->nlev - 1) { or2d_coarse_solve(mg, l); return; }
    for (int s = 0; s < nu1; s++) or2d_smooth(mg, l, omega, smoother);
    or2d_restrict(mg, l);
    memset(mg->dU[l + 1], 0, sizeof(double) * 3 * mg->nx[l + 1] * mg->ny[l + 1]);
    or2d_vcycle(mg, l + 1, omega, nu1, nu2, smoother);
    or2d_prolong(mg, l);
    for (int s = 0; s < nu2; s++) or2d_smooth(mg, l, omega, smoother);
}

void or2d_vcycles(int nx, int ny, int levels, int which, const double *J, const double *rhs, double *dU,
                  int ncycles, double omega, int nu1, int nu2, int smoother)
{
    or2d_mg *mg = or2d_mg_create(nx, ny, levels, which);
    or2d_mg_setup(mg, J);
    memcpy(mg->rhs[0], rhs, sizeof(double) * 3 * nx * ny);
    memcpy(mg->dU[0], dU, sizeof(double) * 3 * nx * ny);
    for (int m = 0; m < ncycles; m++) or2d_vcycle(mg, 0, omega, nu1, nu2, smoother);
    memcpy(dU, mg->dU[0], sizeof(double) * 3 * nx * ny);
    or2d_mg_free(mg);
}

void or2d_smooth_only(int nx, int ny, int which, const double *J, const double *rhs, double *dU,
                      int iters, double omega, int smoother)
{
    or2d_mg *mg = or2d_mg_create(nx, ny, 1, which);
    or2d_mg_setup(mg, J);
    memcpy(mg->rhs[0], rhs, sizeof(double) * 3 * nx * ny);
    memcpy(mg->dU[0], dU, sizeof(double) * 3 * nx * ny);
    for (int s = 0; s < iters; s++) or2d_smooth(mg, 0, omega, smoother);
    memcpy(dU, mg->dU[0], sizeof(double) * 3 * nx * ny);
    or2d_mg_free(mg);
}

/* Algorithm 1 with nu3 V-cycles per step; U is [3][Ny][Nx]. */
int or2d_newton_solve(const or2d_prob *p, const or2d_params *pp, double *U, double *hist, int max_hist,
                      double *res_out)
{
    int Nx = p->Nx, Ny = p->Ny, n = Nx * Ny;
    double *R = malloc(sizeof(double) * 3 * n);
    double *rn = malloc(sizeof(double) * n);
    int off[21][2];
    int nb = or2d_stencil(pp->stencil, off);
    double *J = malloc(sizeof(double) * (size_t)n * nb * 9);
    or2d_mg *mg = or2d_mg_create(Nx, Ny, pp->levels, pp->stencil);
    double res = or2d_residual(p, U, R, rn);
    int it = 0;
    do {
        or2d_jacobian(p, U, R, rn, pp->eps, pp->alpha, pp->stencil, J);
        or2d_mg_setup(mg, J);
        for (int j = 0; j < Ny; j++)
            for (int i = 0; i < Nx; i++)
                for (int c = 0; c < 3; c++) mg->rhs[0][(j * Nx + i) * 3 + c] = R[UIDX(p, c, i, j)];
        memset(mg->dU[0], 0, sizeof(double) * 3 * n);
        for (int m = 0; m < pp->nu3; m++) or2d_vcycle(mg, 0, pp->omega, pp->nu1, pp->nu2, pp->smoother);
        for (int j = 0; j < Ny; j++)
            for (int i = 0; i < Nx; i++)
                for (int c = 0; c < 3; c++)
                    U[UIDX(p, c, i, j)] = U[UIDX(p, c, i, j)] + pp->tau * mg->dU[0][(j * Nx + i) * 3 + c];
        res = or2d_residual(p, U, R, rn);
        if (hist && it < max_hist) hist[it] = res;
        it++;
        if (!(res == res)) break;
    } while (!(res < pp->tol) && it < pp->n_max);
    if (res_out) *res_out = res;
    or2d_mg_free(mg);
    free(R); free(rn); free(J);
    return it;
}

/* ---- nested iteration: Appendix A in two dimensions (eq. A.3) ------------------------------ */

/* One line of eq. (A.2): the averages over the two halves of each of n coarse cells of the
 * quadratic (A.1) through the cell and its two neighbours (reading: the first and last cell use
 * the quadratic centred one cell inward), read with stride `is` and written with stride `os`. */
static void a2_line(int n, const double *u, int is, double *v, int os)
{
    for (int j = 0; j < n; j++) {
        if (j >= 1 && j <= n - 2) {
            v[(2 * j) * os] = u[(j - 1) * is] / 8.0 + u[j * is] - u[(j + 1) * is] / 8.0;
            v[(2 * j + 1) * os] = -u[(j - 1) * is] / 8.0 + u[j * is] + u[(j + 1) * is] / 8.0;
        } else {
            const int k = j == 0 ? 1 : n - 2;
            /* P(xi) = u_k + a xi + b (xi^2 - 1/12), xi in coarse cell widths from the centre of k */
            const double a = (u[(k + 1) * is] - u[(k - 1) * is]) / 2.0;
            const double b = (u[(k - 1) * is] - 2.0 * u[k * is] + u[(k + 1) * is]) / 2.0;
            for (int half = 0; half < 2; half++) {
                const double lo = (double)(j - k) - 0.5 + 0.5 * half, hi = lo + 0.5;
                const double m1 = (lo + hi) / 2.0;                      /* mean of xi   */
                const double m2 = (lo * lo + lo * hi + hi * hi) / 3.0;  /* mean of xi^2 */
                v[(2 * j + half) * os] = u[k * is] + a * m1 + b * (m2 - 1.0 / 12.0);
            }
        }
    }
}

/* Fine cell averages of the polynomial of eq. (A.3) from a coarse state [3][nyc][nxc] to
 * [3][2 nyc][2 nxc].  P is the tensor product of the one-dimensional quadratics (A.1), so its
 * average over a quarter of a coarse cell is the x average of (A.2) taken in each of the three
 * coarse rows and then combined along y with the same weights: first every coarse row is
 * refined in x, then every fine column in y.  nxc, nyc >= 3. */
void or2d_interp_a3(int nxc, int nyc, const double *Uc, double *Uf)
{
    const int nxf = 2 * nxc, nyf = 2 * nyc;
    double *t = malloc(sizeof(double) * (size_t)nyc * nxf);
    for (int c = 0; c < 3; c++) {
        const double *u = Uc + (size_t)c * nyc * nxc;
        double *v = Uf + (size_t)c * nyf * nxf;
        for (int j = 0; j < nyc; j++) a2_line(nxc, u + (size_t)j * nxc, 1, t + (size_t)j * nxf, 1);
        for (int i = 0; i < nxf; i++) a2_line(nyc, t + i, nxf, v + i, nxf);
    }
    free(t);
}
