/*
 * CPU ORACLE -- test infrastructure only.
 *
 * A plain, slow, single-threaded FP64 implementation of the one-dimensional high-order
 * Newton multigrid method (NMGM) for the steady quasi-1D shallow water equations, written
 * step by step from the paper (Hu, Li, Wang, Wang: "A high-order Newton multigrid method with
 * a simplified Jacobian for steady-state shallow water equations").  It exists to check the
 * GPU path: only the test suite, the smoke check and the benchmark's CPU-baseline leg call
 * it.  It shares no code, header or constant table with the GPU library.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math; no FMA contraction), so every
 * expression is evaluated exactly as written.
 *
 * Conventions.  Cells are numbered j = 0..N-1 (the paper uses 1..N).  Conserved variables are
 * U = (H, Q) = (sigma h, sigma h u) (eq. 3-4), stored component-major: U[c*N + j].  Two ghost
 * cells per side complete the five-cell stencil of eq. (10); they are not unknowns (the text
 * after eq. 16 sets J = 0 outside the grid).  The Jacobian is stored as blocks
 * J[((j*nb + b)*2 + l)*2 + m], block b <-> column cell i = j + b - nb/2, entry (l, m) =
 * d R_j^l / d U_i^m.
 *
 * Readings where the paper is silent or garbled (each is listed in the design notes):
 *  R1  WENO3 linear weights: the printed d_r / d~_r labels of eq. (8) give only second order
 *      with the printed candidates; the third-order pairing is used: U+_{j-1/2} takes 1/3 on
 *      T0 = {j, j+1} and 2/3 on T1 = {j-1, j}; U-_{j+1/2} takes 2/3 on T0 and 1/3 on T1.
 *  R2  HLL wave speeds (section 3.1 names HLL without speeds): Davis bounds
 *      S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R), c = sqrt(g h).
 *  R3  Ghost cells (not specified): DISCHARGE side sets Q = q and copies H (or sets
 *      H = sigma h when the boundary cell is supercritical and h > 0 is given); DEPTH side
 *      sets H = sigma h when the boundary cell is subcritical, else copies H, and copies Q;
 *      EXTRAP copies; WALL mirrors with Q negated.  sigma is the width at the boundary face.
 *      Ghosts are recomputed from the (perturbed) state inside every residual evaluation.
 *  R4  Finite-difference perturbation (eq. 12) is absolute and the same for every component.
 *  R5  Multicolour block SOR: colour j mod C (C = 2 for three-block rows, 3 for five-block
 *      rows); one symmetric step sweeps colours 0..C-1 then C-1..0.  The paper's
 *      lexicographic forward+backward sweep (eq. 19) is kept as an option.
 *  R6  The coarsest system is solved by dense Gaussian elimination with partial pivoting.
 *  R7  Optional surface reconstruction (recon = 1, constant width only; not the paper's scheme,
 *      which is not well balanced): WENO3 runs on the surface eta = H + zbar (zbar the cell
 *      average of the bottom), face depths are eta -/+ minus the bottom at the face, and the
 *      source integral -g int h b_x over the cell is split exactly as
 *        -g [ int (eta_h - eta_j) b_x  +  eta_j (b_{j+1/2} - b_{j-1/2})  -  (b_{j+1/2}^2 - b_{j-1/2}^2) / 2 ],
 *      eta_h the cubic through the four face values of eta (two-point Gauss rule for the first
 *      integral), eta_j = H_j + zbar_j.  A still surface (eta constant, Q = 0) then has R = 0 up
 *      to rounding on any bottom.  Ghosts copy eta where R3 copies H (H_g = H_src + zbar_src -
 *      zbar_g); imposed depths stay H = h.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_BC_DISCHARGE 0
#define OR_BC_DEPTH 1
#define OR_BC_EXTRAP 2
#define OR_BC_WALL 3

typedef struct {
    int N;                  /* number of cells */
    double dx;              /* uniform cell size */
    double g;               /* gravity */
    const double *sig_face; /* [N+1] width at face x_{j-1/2}, j = 0..N */
    const double *sig_gp;   /* [2N]  width at the two Gauss points of cell j: 2j (left), 2j+1 */
    const double *sigx_gp;  /* [2N]  d sigma / dx at the Gauss points */
    const double *bx_gp;    /* [2N]  d b / dx at the Gauss points */
    int bc_kind[2];         /* left, right */
    double bc_q[2];
    double bc_h[2];
    int recon;              /* 0: reconstruct H (the paper); 1: reconstruct the surface (R7) */
    const double *z_face;   /* [N+1] bottom at face x_{j-1/2} (recon = 1) */
    const double *z_avg;    /* [N+4] cell averages of the bottom, cells -2..N+1 (recon = 1) */
} or1d_prob;

typedef struct {
    double alpha, tau, eps, omega, tol;
    int nu1, nu2, nu3, n_max;
    int levels;     /* L + 1 */
    int nb;         /* 3 (simplified J3) or 5 (full J5) */
    int smoother;   /* 0 multicolour, 1 lexicographic forward+backward */
    int linear;     /* 0: nu3 V-cycles (Algorithm 1 with Algorithm 2); 1: Newton-SOR */
    int sor_max;    /* Newton-SOR: at most this many symmetric SOR steps per Newton step */
    double sor_tol; /* ... stopping once the l1 norm of the change of dU falls below this */
} or1d_params;

static const double ZETA = 1e-6; /* WENO epsilon of eq. (8) */

/* ------------------------------------------------------------------------------------ */
/* Boundary ghosts (reading R3).  Ug holds N+4 cells, Ug[(k)*2 + c] with k = j + 2.       */
/* ------------------------------------------------------------------------------------ */

static int subcritical(double H, double Q, double sig, double g)
{
    /* Fr^2 = u^2 / (g h) < 1 with u = Q/H, h = H/sig */
    double h = H / sig;
    double u = Q / H;
    return u * u < g * h;
}

void or1d_fill_ghosts(const or1d_prob *p, const double *U, double *Ug)
{
    int N = p->N;
    for (int j = 0; j < N; j++) {
        Ug[(j + 2) * 2 + 0] = U[j];
        Ug[(j + 2) * 2 + 1] = U[N + j];
    }
    for (int side = 0; side < 2; side++) {
        int b0 = side == 0 ? 0 : N - 1;            /* boundary cell */
        int b1 = side == 0 ? 1 : N - 2;            /* next interior cell (for mirrors) */
        int g0 = side == 0 ? -1 : N;               /* first ghost */
        int g1 = side == 0 ? -2 : N + 1;           /* second ghost */
        double sig = p->sig_face[side == 0 ? 0 : N];
        double H0 = U[b0], Q0 = U[N + b0];
        double H1 = U[b1], Q1 = U[N + b1];
        /* copies carry H, or with the surface reconstruction (R7) the surface H + zbar */
        double c00 = 0.0, c01 = 0.0, c11 = 0.0;   /* zbar_src - zbar_ghost for the copies */
        if (p->recon == 1) {
            c00 = p->z_avg[b0 + 2] - p->z_avg[g0 + 2];
            c01 = p->z_avg[b0 + 2] - p->z_avg[g1 + 2];
            c11 = p->z_avg[b1 + 2] - p->z_avg[g1 + 2];
        }
        double Hg0 = H0 + c00, Qg0 = Q0, Hg1 = H0 + c01, Qg1 = Q0;
        switch (p->bc_kind[side]) {
        case OR_BC_DISCHARGE:
            Qg0 = Qg1 = p->bc_q[side];
            if (!subcritical(H0, Q0, sig, p->g) && p->bc_h[side] > 0.0)
                Hg0 = Hg1 = sig * p->bc_h[side];
            break;
        case OR_BC_DEPTH:
            if (subcritical(H0, Q0, sig, p->g))
                Hg0 = Hg1 = sig * p->bc_h[side];
            break;
        case OR_BC_WALL:
            Hg0 = H0 + c00; Qg0 = -Q0;
            Hg1 = H1 + c11; Qg1 = -Q1;
            break;
        default: /* EXTRAP */
            break;
        }
        Ug[(g0 + 2) * 2 + 0] = Hg0; Ug[(g0 + 2) * 2 + 1] = Qg0;
        Ug[(g1 + 2) * 2 + 0] = Hg1; Ug[(g1 + 2) * 2 + 1] = Qg1;
    }
}

/* ------------------------------------------------------------------------------------ */
/* WENO3 reconstruction, eq. (7)-(8) with reading R1.                                     */
/* ------------------------------------------------------------------------------------ */

/* U+_{j-1/2}: right state at the left face of cell j, from cells j-1, j, j+1 */
double or1d_weno_plus(double um, double u0, double up)
{
    double c0 = 1.5 * u0 - 0.5 * up;          /* candidate on T0 = {j, j+1} */
    double c1 = 0.5 * um + 0.5 * u0;          /* candidate on T1 = {j-1, j} */
    double b0 = (up - u0) * (up - u0);        /* smoothness indicators */
    double b1 = (u0 - um) * (u0 - um);
    double a0 = (1.0 / 3.0) / ((ZETA + b0) * (ZETA + b0));
    double a1 = (2.0 / 3.0) / ((ZETA + b1) * (ZETA + b1));
    double w0 = a0 / (a0 + a1);
    double w1 = a1 / (a0 + a1);
    return w0 * c0 + w1 * c1;
}

/* U-_{j+1/2}: left state at the right face of cell j, from cells j-1, j, j+1 */
double or1d_weno_minus(double um, double u0, double up)
{
    double c0 = 0.5 * u0 + 0.5 * up;          /* candidate on T0 = {j, j+1} */
    double c1 = -0.5 * um + 1.5 * u0;         /* candidate on T1 = {j-1, j} */
    double b0 = (up - u0) * (up - u0);
    double b1 = (u0 - um) * (u0 - um);
    double a0 = (2.0 / 3.0) / ((ZETA + b0) * (ZETA + b0));
    double a1 = (1.0 / 3.0) / ((ZETA + b1) * (ZETA + b1));
    double w0 = a0 / (a0 + a1);
    double w1 = a1 / (a0 + a1);
    return w0 * c0 + w1 * c1;
}

/* ------------------------------------------------------------------------------------ */
/* Physical flux of eq. (4) and the HLL numerical flux (reading R2).                      */
/* ------------------------------------------------------------------------------------ */

void or1d_flux(double H, double Q, double sig, double g, double F[2])
{
    double h = H / sig;
    F[0] = Q;
    F[1] = Q * Q / H + 0.5 * g * sig * h * h;
}

void or1d_hll(const double UL[2], const double UR[2], double sig, double g, double F[2])
{
    double FL[2], FR[2];
    or1d_flux(UL[0], UL[1], sig, g, FL);
    or1d_flux(UR[0], UR[1], sig, g, FR);
    double hL = UL[0] / sig, hR = UR[0] / sig;
    double uL = UL[1] / UL[0], uR = UR[1] / UR[0];
    double cL = sqrt(g * hL), cR = sqrt(g * hR);
    double sl1 = uL - cL, sl2 = uR - cR;
    double sr1 = uL + cL, sr2 = uR + cR;
    double SL = sl1 < sl2 ? sl1 : sl2;
    double SR = sr1 > sr2 ? sr1 : sr2;
    if (SL >= 0.0) {
        F[0] = FL[0]; F[1] = FL[1];
    } else if (SR <= 0.0) {
        F[0] = FR[0]; F[1] = FR[1];
    } else {
        for (int c = 0; c < 2; c++)
            F[c] = (SR * FL[c] - SL * FR[c] + SL * SR * (UR[c] - UL[c])) / (SR - SL);
    }
}

/* ------------------------------------------------------------------------------------ */
/* Source quadrature, eq. (9): two-point Gauss rule on S(U_h), U_h the cubic through the   */
/* reconstructed values at x_{j-3/2}, x_{j-1/2}, x_{j+1/2}, x_{j+3/2}.                     */
/* ------------------------------------------------------------------------------------ */

/* Lagrange weights of the nodes t = -3/2, -1/2, 1/2, 3/2 (in units of dx from x_j),
 * evaluated at the Gauss points t = -1/(2 sqrt 3) (row 0) and +1/(2 sqrt 3) (row 1),
 * straight from the product definition of the Lagrange basis. */
void or1d_cubic_gauss_weights(double Wt[2][4])
{
    const double nodes[4] = {-1.5, -0.5, 0.5, 1.5};
    double tg[2];
    tg[0] = -1.0 / (2.0 * sqrt(3.0));
    tg[1] = 1.0 / (2.0 * sqrt(3.0));
    for (int q = 0; q < 2; q++)
        for (int k = 0; k < 4; k++) {
            double w = 1.0;
            for (int m = 0; m < 4; m++)
                if (m != k)
                    w *= (tg[q] - nodes[m]) / (nodes[k] - nodes[m]);
            Wt[q][k] = w;
        }
}

/* S_j (second component; the first is zero) from the four face values of H. */
double or1d_source(const or1d_prob *p, int j, const double Hf[4])
{
    double Wt[2][4];
    or1d_cubic_gauss_weights(Wt);
    double sum = 0.0;
    for (int q = 0; q < 2; q++) {
        double Hg = Wt[q][0] * Hf[0] + Wt[q][1] * Hf[1] + Wt[q][2] * Hf[2] + Wt[q][3] * Hf[3];
        double sg = p->sig_gp[2 * j + q];
        double hg = Hg / sg;
        double s = 0.5 * p->g * hg * hg * p->sigx_gp[2 * j + q] - p->g * sg * hg * p->bx_gp[2 * j + q];
        sum = sum + s;
    }
    return 0.5 * p->dx * sum;
}

/* ------------------------------------------------------------------------------------ */
/* Local residual, eq. (10): R_j = F(U-_{j+1/2}, U+_{j+1/2}) - F(U-_{j-1/2}, U+_{j-1/2})   */
/* - S_j, from the ghost-extended state.  Not divided by dx.                             */
/* ------------------------------------------------------------------------------------ */

#define UG(k, c) Ug[((k) + 2) * 2 + (c)]

/* R7: the local residual with the surface reconstructed (constant width, sigma = 1) */
static void local_residual_surface(const or1d_prob *p, const double *Ug, int j, double R[2])
{
    double E[5];   /* surface eta = H + zbar on cells j-2..j+2 */
    for (int k = 0; k < 5; k++) E[k] = UG(j - 2 + k, 0) + p->z_avg[j + k];
    double Em_jm = or1d_weno_minus(E[0], E[1], E[2]);   /* eta-_{j-1/2}, from cell j-1 */
    double Ep_jm = or1d_weno_plus(E[1], E[2], E[3]);    /* eta+_{j-1/2}, from cell j */
    double Em_jp = or1d_weno_minus(E[1], E[2], E[3]);   /* eta-_{j+1/2}, from cell j */
    double Ep_jp = or1d_weno_plus(E[2], E[3], E[4]);    /* eta+_{j+1/2}, from cell j+1 */
    double Ep_jmm = or1d_weno_plus(E[0], E[1], E[2]);   /* eta+_{j-3/2}, from cell j-1 */
    double Em_jpp = or1d_weno_minus(E[2], E[3], E[4]);  /* eta-_{j+3/2}, from cell j+1 */
    double zl = p->z_face[j], zr = p->z_face[j + 1];
    double Um_jm[2] = {Em_jm - zl, or1d_weno_minus(UG(j - 2, 1), UG(j - 1, 1), UG(j, 1))};
    double Up_jm[2] = {Ep_jm - zl, or1d_weno_plus(UG(j - 1, 1), UG(j, 1), UG(j + 1, 1))};
    double Um_jp[2] = {Em_jp - zr, or1d_weno_minus(UG(j - 1, 1), UG(j, 1), UG(j + 1, 1))};
    double Up_jp[2] = {Ep_jp - zr, or1d_weno_plus(UG(j, 1), UG(j + 1, 1), UG(j + 2, 1))};
    double Fm[2], Fp[2];
    or1d_hll(Um_jm, Up_jm, 1.0, p->g, Fm);
    or1d_hll(Um_jp, Up_jp, 1.0, p->g, Fp);
    /* the split source of R7 */
    double Wt[2][4];
    or1d_cubic_gauss_weights(Wt);
    double eta_j = E[2];
    double quad = 0.0;
    for (int q = 0; q < 2; q++) {
        double eg = Wt[q][0] * Ep_jmm + Wt[q][1] * Ep_jm + Wt[q][2] * Em_jp + Wt[q][3] * Em_jpp;
        quad = quad + (eg - eta_j) * p->bx_gp[2 * j + q];
    }
    double S = -p->g * (0.5 * p->dx * quad + eta_j * (zr - zl) - 0.5 * (zr * zr - zl * zl));
    R[0] = Fp[0] - Fm[0];
    R[1] = Fp[1] - Fm[1] - S;
}

void or1d_local_residual(const or1d_prob *p, const double *Ug, int j, double R[2])
{
    if (p->recon == 1) {
        local_residual_surface(p, Ug, j, R);
        return;
    }
    double Um_jm[2], Up_jm[2], Um_jp[2], Up_jp[2];  /* U-_{j-1/2}, U+_{j-1/2}, U-_{j+1/2}, U+_{j+1/2} */
    double Hp_jmm, Hm_jpp;                          /* H+_{j-3/2}, H-_{j+3/2} */
    for (int c = 0; c < 2; c++) {
        Um_jm[c] = or1d_weno_minus(UG(j - 2, c), UG(j - 1, c), UG(j, c));     /* from cell j-1 */
        Up_jm[c] = or1d_weno_plus(UG(j - 1, c), UG(j, c), UG(j + 1, c));      /* from cell j */
        Um_jp[c] = or1d_weno_minus(UG(j - 1, c), UG(j, c), UG(j + 1, c));     /* from cell j */
        Up_jp[c] = or1d_weno_plus(UG(j, c), UG(j + 1, c), UG(j + 2, c));      /* from cell j+1 */
    }
    Hp_jmm = or1d_weno_plus(UG(j - 2, 0), UG(j - 1, 0), UG(j, 0));            /* from cell j-1 */
    Hm_jpp = or1d_weno_minus(UG(j, 0), UG(j + 1, 0), UG(j + 2, 0));           /* from cell j+1 */

    double Fm[2], Fp[2];
    or1d_hll(Um_jm, Up_jm, p->sig_face[j], p->g, Fm);
    or1d_hll(Um_jp, Up_jp, p->sig_face[j + 1], p->g, Fp);
    double Hf[4] = {Hp_jmm, Up_jm[0], Um_jp[0], Hm_jpp};
    double S = or1d_source(p, j, Hf);
    R[0] = Fp[0] - Fm[0];
    R[1] = Fp[1] - Fm[1] - S;
}

/* Global residual: R[c*N + j], rn[j] = ||R_j||_1; returns res = (1/N) sum_j ||R_j||_1
 * (Algorithm 1, evaluation of the global residual). */
double or1d_residual(const or1d_prob *p, const double *U, double *R, double *rn)
{
    int N = p->N;
    double *Ug = malloc(sizeof(double) * 2 * (N + 4));
    or1d_fill_ghosts(p, U, Ug);
    double sum = 0.0;
    for (int j = 0; j < N; j++) {
        double Rj[2];
        or1d_local_residual(p, Ug, j, Rj);
        R[j] = Rj[0];
        R[N + j] = Rj[1];
        double n1 = fabs(Rj[0]) + fabs(Rj[1]);
        if (rn) rn[j] = n1;
        sum += n1;
    }
    free(Ug);
    return sum / N;
}

/* ------------------------------------------------------------------------------------ */
/* Finite-difference Jacobian, eq. (12), regularised per eq. (13).  Column (i, m) perturbs */
/* the global state U_i^m by eps (ghosts recomputed), and rows j with |i - j| <= nb/2 take */
/* the forward difference of R_j.  nb = 3 keeps the simplified block-tridiagonal J3 of     */
/* section 3.3; nb = 5 gives the full J5.                                                  */
/* ------------------------------------------------------------------------------------ */

void or1d_jacobian(const or1d_prob *p, const double *U, const double *R, const double *rn,
                   double eps, double alpha, int nb, double *J)
{
    int N = p->N, hw = nb / 2;
    double *Up = malloc(sizeof(double) * 2 * N);
    double *Ug = malloc(sizeof(double) * 2 * (N + 4));
    memcpy(Up, U, sizeof(double) * 2 * N);
    memset(J, 0, sizeof(double) * (size_t)N * nb * 4);
    for (int i = 0; i < N; i++) {
        for (int m = 0; m < 2; m++) {
            double saved = Up[m * N + i];
            Up[m * N + i] = saved + eps;
            or1d_fill_ghosts(p, Up, Ug);
            for (int j = i - hw; j <= i + hw; j++) {
                if (j < 0 || j >= N)
                    continue;
                double Rp[2];
                or1d_local_residual(p, Ug, j, Rp);
                int b = i - j + hw;
                for (int l = 0; l < 2; l++)
                    J[((j * nb + b) * 2 + l) * 2 + m] = (Rp[l] - R[l * N + j]) / eps;
            }
            Up[m * N + i] = saved;
        }
    }
    for (int j = 0; j < N; j++)
        for (int l = 0; l < 2; l++)
            J[((j * nb + hw) * 2 + l) * 2 + l] += alpha * rn[j];
    free(Up);
    free(Ug);
}

/* ------------------------------------------------------------------------------------ */
/* Geometric multigrid, section 3.4.                                                      */
/* Level l has n[l] = N / 2^l cells; level 0 has nb-block rows, coarser levels three.     */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    int nlev;
    int n[32];
    int nb[32];
    double *J[32];    /* blocks as for the fine Jacobian */
    double *Dinv[32]; /* [n][2][2] inverse of the diagonal block */
    double *rhs[32];  /* [n][2]: level equation is  sum_i J_ji dU_i = -rhs_j  */
    double *dU[32];   /* [n][2] */
} or1d_mg;

static void inv2(const double A[4], double B[4])
{
    double det = A[0] * A[3] - A[1] * A[2];
    B[0] = A[3] / det;
    B[1] = -A[1] / det;
    B[2] = -A[2] / det;
    B[3] = A[0] / det;
}

/* eq. (17), operator part: J_{ji,l} = sum_{xi in children(j)} sum_{eta in children(i)} J_{xi eta,l-1}.
 * The coarse stencil is three blocks wide for a fine stencil of three or five blocks. */
void or1d_coarsen(int nf, int nbf, const double *Jf, double *Jc)
{
    int nc = nf / 2, hf = nbf / 2;
    memset(Jc, 0, sizeof(double) * (size_t)nc * 3 * 4);
    for (int j = 0; j < nc; j++)
        for (int bc = 0; bc < 3; bc++) {
            int i = j + bc - 1;
            if (i < 0 || i >= nc)
                continue;
            double *blk = &Jc[(j * 3 + bc) * 4];
            for (int xi = 2 * j; xi <= 2 * j + 1; xi++)
                for (int eta = 2 * i; eta <= 2 * i + 1; eta++) {
                    int bf = eta - xi + hf;
                    if (bf < 0 || bf >= nbf)
                        continue;
                    const double *src = &Jf[(xi * nbf + bf) * 4];
                    for (int e = 0; e < 4; e++)
                        blk[e] = blk[e] + src[e];
                }
        }
}

or1d_mg *or1d_mg_create(int N, int levels, int nb)
{
    or1d_mg *mg = calloc(1, sizeof(or1d_mg));
    mg->nlev = levels;
    for (int l = 0; l < levels; l++) {
        mg->n[l] = N >> l;
        mg->nb[l] = l == 0 ? nb : 3;
        mg->J[l] = calloc((size_t)mg->n[l] * mg->nb[l] * 4, sizeof(double));
        mg->Dinv[l] = calloc((size_t)mg->n[l] * 4, sizeof(double));
        mg->rhs[l] = calloc((size_t)mg->n[l] * 2, sizeof(double));
        mg->dU[l] = calloc((size_t)mg->n[l] * 2, sizeof(double));
    }
    return mg;
}

void or1d_mg_free(or1d_mg *mg)
{
    for (int l = 0; l < mg->nlev; l++) {
        free(mg->J[l]); free(mg->Dinv[l]); free(mg->rhs[l]); free(mg->dU[l]);
    }
    free(mg);
}

/* Load the fine operator and build every coarse operator and diagonal inverse.  The coarse
 * operators do not depend on dU, so building them once per Newton step gives the same values
 * as constructing them inside every cycle (Algorithm 2, coarse-level correction). */
void or1d_mg_setup(or1d_mg *mg, const double *Jfine)
{
    memcpy(mg->J[0], Jfine, sizeof(double) * (size_t)mg->n[0] * mg->nb[0] * 4);
    for (int l = 1; l < mg->nlev; l++)
        or1d_coarsen(mg->n[l - 1], mg->nb[l - 1], mg->J[l - 1], mg->J[l]);
    for (int l = 0; l < mg->nlev; l++) {
        int nb = mg->nb[l], hw = nb / 2;
        for (int j = 0; j < mg->n[l]; j++)
            inv2(&mg->J[l][(j * nb + hw) * 4], &mg->Dinv[l][j * 4]);
    }
}

double *or1d_mg_level_J(or1d_mg *mg, int l) { return mg->J[l]; }
double *or1d_mg_level_Dinv(or1d_mg *mg, int l) { return mg->Dinv[l]; }
double *or1d_mg_level_rhs(or1d_mg *mg, int l) { return mg->rhs[l]; }
double *or1d_mg_level_dU(or1d_mg *mg, int l) { return mg->dU[l]; }

/* One block SOR update of cell j, eq. (19):
 * dU_j <- (1-w) dU_j - w J_jj^{-1} (R_j + sum_{i != j} J_ji dU_i). */
static void sor_update(const or1d_mg *mg, int l, int j, double omega)
{
    int n = mg->n[l], nb = mg->nb[l], hw = nb / 2;
    const double *J = mg->J[l];
    double *dU = mg->dU[l];
    double r0 = mg->rhs[l][2 * j], r1 = mg->rhs[l][2 * j + 1];
    for (int b = 0; b < nb; b++) {
        int i = j + b - hw;
        if (b == hw || i < 0 || i >= n)
            continue;
        const double *blk = &J[(j * nb + b) * 4];
        r0 = r0 + (blk[0] * dU[2 * i] + blk[1] * dU[2 * i + 1]);
        r1 = r1 + (blk[2] * dU[2 * i] + blk[3] * dU[2 * i + 1]);
    }
    const double *D = &mg->Dinv[l][j * 4];
    double t0 = D[0] * r0 + D[1] * r1;
    double t1 = D[2] * r0 + D[3] * r1;
    dU[2 * j] = (1.0 - omega) * dU[2 * j] - omega * t0;
    dU[2 * j + 1] = (1.0 - omega) * dU[2 * j + 1] - omega * t1;
}

/* One symmetric smoothing step on level l (reading R5). */
void or1d_smooth(or1d_mg *mg, int l, double omega, int smoother)
{
    int n = mg->n[l];
    if (smoother == 1) {
        for (int j = 0; j < n; j++) sor_update(mg, l, j, omega);
        for (int j = n - 1; j >= 0; j--) sor_update(mg, l, j, omega);
        return;
    }
    int C = mg->nb[l] == 5 ? 3 : 2;
    for (int c = 0; c < C; c++)
        for (int j = c; j < n; j += C) sor_update(mg, l, j, omega);
    for (int c = C - 1; c >= 0; c--)
        for (int j = c; j < n; j += C) sor_update(mg, l, j, omega);
}

/* Coarsest level: solve sum_i J_ji dU_i = -rhs_j by dense Gaussian elimination with
 * partial pivoting (reading R6). */
void or1d_coarse_solve(or1d_mg *mg, int l)
{
    int n = mg->n[l], nb = mg->nb[l], hw = nb / 2, M = 2 * n;
    double *A = calloc((size_t)M * M, sizeof(double));
    double *x = calloc(M, sizeof(double));
    for (int j = 0; j < n; j++)
        for (int b = 0; b < nb; b++) {
            int i = j + b - hw;
            if (i < 0 || i >= n)
                continue;
            for (int r = 0; r < 2; r++)
                for (int c = 0; c < 2; c++)
                    A[(2 * j + r) * M + 2 * i + c] = mg->J[l][((j * nb + b) * 2 + r) * 2 + c];
        }
    for (int r = 0; r < M; r++)
        x[r] = -mg->rhs[l][r];
    for (int k = 0; k < M; k++) {
        int piv = k;
        for (int r = k + 1; r < M; r++)
            if (fabs(A[r * M + k]) > fabs(A[piv * M + k]))
                piv = r;
        if (piv != k) {
            for (int c = 0; c < M; c++) {
                double t = A[k * M + c]; A[k * M + c] = A[piv * M + c]; A[piv * M + c] = t;
            }
            double t = x[k]; x[k] = x[piv]; x[piv] = t;
        }
        for (int r = k + 1; r < M; r++) {
            double f = A[r * M + k] / A[k * M + k];
            if (f == 0.0)
                continue;
            for (int c = k; c < M; c++)
                A[r * M + c] -= f * A[k * M + c];
            x[r] -= f * x[k];
        }
    }
    for (int k = M - 1; k >= 0; k--) {
        double s = x[k];
        for (int c = k + 1; c < M; c++)
            s -= A[k * M + c] * x[c];
        x[k] = s / A[k * M + k];
    }
    memcpy(mg->dU[l], x, sizeof(double) * M);
    free(A);
    free(x);
}

/* eq. (17), right-hand side: rhs_{j,l+1} = sum_{xi in children(j)} (rhs_xi + sum_eta J_{xi eta} dU_eta). */
void or1d_restrict(or1d_mg *mg, int l)
{
    int n = mg->n[l], nb = mg->nb[l], hw = nb / 2;
    const double *J = mg->J[l], *dU = mg->dU[l], *rhs = mg->rhs[l];
    double *rc = mg->rhs[l + 1];
    for (int jc = 0; jc < mg->n[l + 1]; jc++) {
        double s0 = 0.0, s1 = 0.0;
        for (int xi = 2 * jc; xi <= 2 * jc + 1; xi++) {
            double a0 = rhs[2 * xi], a1 = rhs[2 * xi + 1];
            for (int b = 0; b < nb; b++) {
                int eta = xi + b - hw;
                if (eta < 0 || eta >= n)
                    continue;
                const double *blk = &J[(xi * nb + b) * 4];
                a0 = a0 + (blk[0] * dU[2 * eta] + blk[1] * dU[2 * eta + 1]);
                a1 = a1 + (blk[2] * dU[2 * eta] + blk[3] * dU[2 * eta + 1]);
            }
            s0 = s0 + a0;
            s1 = s1 + a1;
        }
        rc[2 * jc] = s0;
        rc[2 * jc + 1] = s1;
    }
}

/* eq. (18): dU_{i,l} += dU_{j,l+1} for i = 2j, 2j+1. */
void or1d_prolong(or1d_mg *mg, int l)
{
    double *df = mg->dU[l];
    const double *dc = mg->dU[l + 1];
    for (int jc = 0; jc < mg->n[l + 1]; jc++)
        for (int k = 0; k < 2; k++)
            for (int c = 0; c < 2; c++)
                df[2 * (2 * jc + k) + c] += dc[2 * jc + c];
}

/* Algorithm 2: one V-cycle on level l, starting from the current mg->dU[l]. */
void or1d_vcycle(or1d_mg *mg, int l, double omega, int nu1, int nu2, int smoother)
{
    if (l == mg->nlev - 1) {
        or1d_coarse_solve(mg, l);
        return;
    }
    for (int s = 0; s < nu1; s++)
        or1d_smooth(mg, l, omega, smoother);
    or1d_restrict(mg, l);
    memset(mg->dU[l + 1], 0, sizeof(double) * 2 * mg->n[l + 1]);
    or1d_vcycle(mg, l + 1, omega, nu1, nu2, smoother);
    or1d_prolong(mg, l);
    for (int s = 0; s < nu2; s++)
        or1d_smooth(mg, l, omega, smoother);
}

/* ------------------------------------------------------------------------------------ */
/* Algorithm 1 with the linear system (13) solved by nu3 V-cycles from dU = 0.            */
/* U (component-major [2][N]) is the initial guess on entry and the result on exit.       */
/* Returns the number of Newton iterations; hist[n] = res after iteration n+1.            */
/* ------------------------------------------------------------------------------------ */

int or1d_newton_solve(const or1d_prob *p, const or1d_params *pp, double *U, double *hist, int max_hist,
                      double *res_out)
{
    int N = p->N, nb = pp->nb;
    double *R = malloc(sizeof(double) * 2 * N);
    double *rn = malloc(sizeof(double) * N);
    double *J = malloc(sizeof(double) * (size_t)N * nb * 4);
    or1d_mg *mg = or1d_mg_create(N, pp->linear == 1 ? 1 : pp->levels, nb);
    double res = or1d_residual(p, U, R, rn);
    int n = 0;
    do {
        or1d_jacobian(p, U, R, rn, pp->eps, pp->alpha, nb, J);
        or1d_mg_setup(mg, J);
        for (int j = 0; j < N; j++) {
            mg->rhs[0][2 * j] = R[j];
            mg->rhs[0][2 * j + 1] = R[N + j];
        }
        memset(mg->dU[0], 0, sizeof(double) * 2 * N);
        if (pp->linear == 1) {
            /* Newton-SOR (section 5.1.1, the reference solver of Table 2): the multigrid
             * iteration replaced by symmetric block SOR steps on the grid itself, stopped when
             * the l1 norm of the change between two successive iterates falls below sor_tol or
             * after sor_max steps (reading: the l1 norm sums |change| over all cells and both
             * components) */
            double *old = malloc(sizeof(double) * 2 * N);
            for (int k = 0; k < pp->sor_max; k++) {
                memcpy(old, mg->dU[0], sizeof(double) * 2 * N);
                or1d_smooth(mg, 0, pp->omega, pp->smoother);
                double var = 0.0;
                for (int e = 0; e < 2 * N; e++) var += fabs(mg->dU[0][e] - old[e]);
                if (var < pp->sor_tol) break;
            }
            free(old);
        } else {
            for (int m = 0; m < pp->nu3; m++)
                or1d_vcycle(mg, 0, pp->omega, pp->nu1, pp->nu2, pp->smoother);
        }
        for (int j = 0; j < N; j++) {
            U[j] = U[j] + pp->tau * mg->dU[0][2 * j];
            U[N + j] = U[N + j] + pp->tau * mg->dU[0][2 * j + 1];
        }
        res = or1d_residual(p, U, R, rn);
        if (hist && n < max_hist)
            hist[n] = res;
        n++;
        if (!(res == res))  /* NaN: stop */
            break;
    } while (!(res < pp->tol) && n < pp->n_max);
    if (res_out) *res_out = res;
    or1d_mg_free(mg);
    free(R); free(rn); free(J);
    return n;
}

/* One V-cycle solve of J dU = -rhs for tests: fine operator J (nb-block rows), rhs and dU in
 * [n][2] interleaved layout; ncycles V-cycles starting from dU as given. */
void or1d_vcycles(int N, int levels, int nb, const double *J, const double *rhs, double *dU,
                  int ncycles, double omega, int nu1, int nu2, int smoother)
{
    or1d_mg *mg = or1d_mg_create(N, levels, nb);
    or1d_mg_setup(mg, J);
    memcpy(mg->rhs[0], rhs, sizeof(double) * 2 * N);
    memcpy(mg->dU[0], dU, sizeof(double) * 2 * N);
    for (int m = 0; m < ncycles; m++)
        or1d_vcycle(mg, 0, omega, nu1, nu2, smoother);
    memcpy(dU, mg->dU[0], sizeof(double) * 2 * N);
    or1d_mg_free(mg);
}

/* Smoothing only (no coarse correction), for tests of the smoother's fixed point. */
void or1d_smooth_only(int N, int nb, const double *J, const double *rhs, double *dU, int steps,
                      double omega, int smoother)
{
    or1d_mg *mg = or1d_mg_create(N, 1, nb);
    or1d_mg_setup(mg, J);
    memcpy(mg->rhs[0], rhs, sizeof(double) * 2 * N);
    memcpy(mg->dU[0], dU, sizeof(double) * 2 * N);
    for (int s = 0; s < steps; s++)
        or1d_smooth(mg, 0, omega, smoother);
    memcpy(dU, mg->dU[0], sizeof(double) * 2 * N);
    or1d_mg_free(mg);
}

/* Appendix A, eq. (A.1)-(A.2): initial cell averages of the level-l grid from the coarser
 * level-(l+1) solution (Algorithm 3, step 9).  Uc is [2][nc], Uf is [2][2 nc]; children 2j and
 * 2j+1 (0-based) of coarse cell j.  Interior cells take eq. (A.2) as printed.  Reading (the
 * appendix is silent at the ends): the first and last coarse cells take the quadratic (A.1)
 * centred one cell inward, averaged over their two halves (still conservative and exact for
 * quadratics).  Needs nc >= 3. */
void or1d_interp_a2(int nc, const double *Uc, double *Uf)
{
    const int nf = 2 * nc;
    for (int c = 0; c < 2; c++) {
        const double *u = Uc + (size_t)c * nc;
        double *v = Uf + (size_t)c * nf;
        for (int j = 0; j < nc; j++) {
            if (j >= 1 && j <= nc - 2) {
                v[2 * j] = u[j - 1] / 8.0 + u[j] - u[j + 1] / 8.0;
                v[2 * j + 1] = -u[j - 1] / 8.0 + u[j] + u[j + 1] / 8.0;
            } else {
                const int k = j == 0 ? 1 : nc - 2;
                /* P(xi) = u_k + a xi + b (xi^2 - 1/12), xi = (x - x_k) / dx_coarse */
                const double a = (u[k + 1] - u[k - 1]) / 2.0;
                const double b = (u[k - 1] - 2.0 * u[k] + u[k + 1]) / 2.0;
                for (int half = 0; half < 2; half++) {
                    const double lo = (double)(j - k) - 0.5 + 0.5 * half, hi = lo + 0.5;
                    const double m1 = (lo + hi) / 2.0;                      /* mean of xi   */
                    const double m2 = (lo * lo + lo * hi + hi * hi) / 3.0;  /* mean of xi^2 */
                    v[2 * j + half] = u[k] + a * m1 + b * (m2 - 1.0 / 12.0);
                }
            }
        }
    }
}
