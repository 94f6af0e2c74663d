// 1D finite-volume WENO residual (section 3.1, eq. 5-10) and its finite-difference block
// Jacobian (section 3.2-3.3, eq. 12-13) for gfx950.
//
// One thread per cell; a 256-cell tile stages U (+2 halo cells per side) in LDS so that the
// five-cell stencil of eq. (10) is read from HBM once.  The residual kernel evaluates R_j per
// thread; the Jacobian kernel evaluates one face per thread (the unperturbed state and every
// column perturbation that reaches it) and assembles each row from its faces, taken from the
// neighbouring lanes (rows within two cells of a side re-evaluate their own stencil with
// ghosts).  FP64 division is the costly operation here (a reciprocal
// and several dependent FMAs each), so the formulas are evaluated in algebraically equal forms
// with few divisions: one per WENO3 reconstruction (the normalised weights combined over a
// common denominator), one reciprocal per depth and wave-speed difference in the HLL flux,
// reciprocals of the widths once per cell and of the perturbation once per launch.  Those
// divisions and reciprocals use the hardware reciprocal refined by Newton-Raphson steps instead
// of the fully IEEE-rounded sequence (their operands are well scaled), so a quotient may differ
// from the correctly rounded one in its last bit.  The result agrees with the printed forms to
// rounding.
//
// This file's kernels are bound by FP64 arithmetic, so a product added to another term within
// one expression is contracted into a single fused multiply-add (the library's other files keep
// contraction off).  Contraction follows the source expressions alone, so every kernel that
// evaluates a residual here rounds it the same way.
#include "nmg_common.h"

#pragma clang fp contract(on)

namespace nmg {

// a / b within about an ulp for the well-scaled operands of this file: the hardware's approximate
// reciprocal refined by two Newton-Raphson steps x <- x + x (1 - b x), then the quotient a x
// corrected once by its residual a - b q (no range scaling: |b| stays far from the overflow
// and denormal limits here)
__device__ __forceinline__ double qrcp(double b)
{
    double x = __builtin_amdgcn_rcp(b);
    x = fma(fma(-b, x, 1.0), x, x);
    x = fma(fma(-b, x, 1.0), x, x);
    return x;
}

__device__ __forceinline__ double qdiv(double a, double b)
{
    const double x = qrcp(b);
    const double q = a * x;
    return fma(fma(-b, q, a), x, q);
}

// sqrt(a) for a positive normal a (here g h at a face, h > 0): the hardware's reciprocal square
// root r refined by the coupled Goldschmidt iteration on g ~ a r and h ~ r / 2, then two residual
// corrections g += (a - g^2) h.  These are the operations of the IEEE-rounded square root without
// its scaling of tiny arguments and its handling of zero and infinity, which such an a never needs.
__device__ __forceinline__ double qsqrt(double a)
{
    const double r = __builtin_amdgcn_rsq(a);
    double g = a * r, h = r * 0.5;
    const double e = fma(-h, g, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    double d = fma(-g, g, a);
    g = fma(d, h, g);
    d = fma(-g, g, a);
    return fma(d, h, g);
}

// ---- WENO3 reconstruction (eq. 7-8) ----------------------------------------------------
// Linear weights paired for third order: the central two-cell candidate takes 2/3 (the
// printed d_r labels of eq. 8 are swapped; with them the scheme is second order).

__device__ __forceinline__ double weno_plus(double um, double u0, double up)
{
    // right state U+_{j-1/2} at the left face of cell j: candidates T0 = {j, j+1} (weight 1/3)
    // and T1 = {j-1, j} (2/3); w_r = alpha_r / (alpha_0 + alpha_1) with
    // alpha_r = d_r / (zeta + beta_r)^2, combined over the common denominator
    const double c0 = 1.5 * u0 - 0.5 * up;
    const double c1 = 0.5 * um + 0.5 * u0;
    const double z0 = kZeta + (up - u0) * (up - u0);
    const double z1 = kZeta + (u0 - um) * (u0 - um);
    const double e0 = z0 * z0, e1 = z1 * z1;
    return qdiv(e1 * c0 + 2.0 * (e0 * c1), e1 + 2.0 * e0);
}

__device__ __forceinline__ double weno_minus(double um, double u0, double up)
{
    // left state U-_{j+1/2} at the right face of cell j: T0 = {j, j+1} (2/3), T1 = {j-1, j} (1/3)
    const double c0 = 0.5 * u0 + 0.5 * up;
    const double c1 = -0.5 * um + 1.5 * u0;
    const double z0 = kZeta + (up - u0) * (up - u0);
    const double z1 = kZeta + (u0 - um) * (u0 - um);
    const double e0 = z0 * z0, e1 = z1 * z1;
    return qdiv(2.0 * (e1 * c0) + e0 * c1, 2.0 * e1 + e0);
}

// ---- HLL flux for eq. (4) with Davis wave-speed bounds ----------------------------------

__device__ __forceinline__ void hll(double HL, double QL, double HR, double QR, double sig,
                                    double isig, double g, double &F0, double &F1)
{
    // sig: width at the face, isig = 1 / sig
    const double iHL = qrcp(HL), iHR = qrcp(HR);
    const double hl = HL * isig, hr = HR * isig;
    const double uL = QL * iHL, uR = QR * iHR;
    const double FL0 = QL, FL1 = QL * uL + 0.5 * g * sig * hl * hl;
    const double FR0 = QR, FR1 = QR * uR + 0.5 * g * sig * hr * hr;
    const double cL = qsqrt(g * hl), cR = qsqrt(g * hr);
    const double sl1 = uL - cL, sl2 = uR - cR;
    const double sr1 = uL + cL, sr2 = uR + cR;
    const double SL = sl1 < sl2 ? sl1 : sl2;
    const double SR = sr1 > sr2 ? sr1 : sr2;
    // the HLL average is formed whatever the wave speeds (SR > SL since the celerities are
    // positive) and the upwind cases select: no branch, so that independent fluxes interleave.
    // The empty asm statement (no instruction) takes the average as its operand, which keeps
    // the compiler from moving its evaluation into a branch of its own.
    const double iw = qrcp(SR - SL);
    double G0 = (SR * FL0 - SL * FR0 + SL * SR * (HR - HL)) * iw;
    double G1 = (SR * FL1 - SL * FR1 + SL * SR * (QR - QL)) * iw;
    asm("" : "+v"(G0), "+v"(G1));
    F0 = SL >= 0.0 ? FL0 : (SR <= 0.0 ? FR0 : G0);
    F1 = SL >= 0.0 ? FL1 : (SR <= 0.0 ? FR1 : G1);
}

// Lagrange weights of the cubic through x_{j-3/2}, x_{j-1/2}, x_{j+1/2}, x_{j+3/2} at the two
// Gauss points x_j -/+ dx/(2 sqrt 3) (eq. 9), from the product form of the basis.
struct CubicGauss {
    double w[2][4];
    __device__ CubicGauss()
    {
        const double t[4] = {-1.5, -0.5, 0.5, 1.5};
        const double tg0 = -1.0 / (2.0 * sqrt(3.0));
        const double tg1 = 1.0 / (2.0 * sqrt(3.0));
#pragma unroll
        for (int q = 0; q < 2; q++) {
            double x = q == 0 ? tg0 : tg1;
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

// Geometry of one cell: faces j-1/2, j+1/2 and the two Gauss points.
struct CellGeom {
    double sfm, sfp, isfm, isfp;      // widths at the faces and their reciprocals
    double sg[2], isg[2], sxg[2], bxg[2];
    double zfm, zfp;                  // bottom at the faces (surface reconstruction)
};

// a load that is this data's last use in the step (STREAM): the non-temporal hint leaves the
// memory-side cache to what the next launch re-reads
template <bool STREAM>
__device__ __forceinline__ double ldg(const double *p)
{
    if (STREAM) return __builtin_nontemporal_load(p);
    return *p;
}

// SURF: the surface reconstruction (constant width 1): the widths are not read, the bottom at
// the faces is
template <bool SURF, bool STREAM = false>
__device__ __forceinline__ CellGeom load_geom(const Inst1D &I, int j)
{
    CellGeom G;
    if (SURF) {
        G.sfm = G.sfp = G.isfm = G.isfp = 1.0;
        G.zfm = ldg<STREAM>(&I.z_face[j]);
        G.zfp = ldg<STREAM>(&I.z_face[j + 1]);
#pragma unroll
        for (int q = 0; q < 2; q++) {
            G.sg[q] = G.isg[q] = 1.0;
            G.sxg[q] = 0.0;
            G.bxg[q] = ldg<STREAM>(&I.bx_gp[2 * j + q]);
        }
        return G;
    }
    G.zfm = G.zfp = 0.0;
    G.sfm = ldg<STREAM>(&I.sig_face[j]);
    G.sfp = ldg<STREAM>(&I.sig_face[j + 1]);
    G.isfm = qrcp(G.sfm);
    G.isfp = qrcp(G.sfp);
#pragma unroll
    for (int q = 0; q < 2; q++) {
        G.sg[q] = ldg<STREAM>(&I.sig_gp[2 * j + q]);
        G.isg[q] = qrcp(G.sg[q]);
        G.sxg[q] = ldg<STREAM>(&I.sigx_gp[2 * j + q]);
        G.bxg[q] = ldg<STREAM>(&I.bx_gp[2 * j + q]);
    }
    return G;
}

__device__ __forceinline__ bool subcrit(double H, double Q, double sig, double g)
{
    double h = H / sig;
    double u = Q / H;
    return u * u < g * h;
}

// Boundary ghosts from the boundary cell (c0) and its neighbour (c1): first and second ghost.
// SURF: a copy carries the surface H + zbar, so the copied H gains c00, c01 or c11 (zbar of
// the source cell minus zbar of the ghost)
template <bool SURF>
__device__ __forceinline__ void ghost_pair(int kind, double q, double hb, double sig, double g,
                                           double H0, double Q0, double H1, double Q1,
                                           double c00, double c01, double c11,
                                           double &Hg0, double &Qg0, double &Hg1, double &Qg1)
{
    Hg0 = SURF ? H0 + c00 : H0; Qg0 = Q0; Hg1 = SURF ? H0 + c01 : H0; Qg1 = Q0;
    if (kind == NMG_BC_DISCHARGE) {
        Qg0 = q; Qg1 = q;
        if (!subcrit(H0, Q0, sig, g) && hb > 0.0) { Hg0 = sig * hb; Hg1 = sig * hb; }
    } else if (kind == NMG_BC_DEPTH) {
        if (subcrit(H0, Q0, sig, g)) { Hg0 = sig * hb; Hg1 = sig * hb; }
    } else if (kind == NMG_BC_WALL) {
        Hg0 = SURF ? H0 + c00 : H0; Qg0 = -Q0; Hg1 = SURF ? H1 + c11 : H1; Qg1 = -Q1;
    }
}

// Fill the ghost entries of a stencil (cells j-2..j+2 at positions 0..4) from its own interior
// entries, so that ghosts follow any perturbation of the boundary cells.
template <bool SURF>
__device__ __forceinline__ void stencil_ghosts(double H[5], double Q[5], int j, const Inst1D &I)
{
    const int N = I.N;
    if (j < 2) {
        const int p0 = 2 - j;  // position of cell 0
        double Hg0, Qg0, Hg1, Qg1;
        double H0 = p0 == 1 ? H[1] : H[2], Q0 = p0 == 1 ? Q[1] : Q[2];
        double H1 = p0 == 1 ? H[2] : H[3], Q1 = p0 == 1 ? Q[2] : Q[3];
        // z_avg holds cells -2..N+1: cell k at k + 2
        const double c00 = SURF ? I.z_avg[2] - I.z_avg[1] : 0.0;
        const double c01 = SURF ? I.z_avg[2] - I.z_avg[0] : 0.0;
        const double c11 = SURF ? I.z_avg[3] - I.z_avg[0] : 0.0;
        ghost_pair<SURF>(I.bc_kind[0], I.bc_q[0], I.bc_h[0], SURF ? 1.0 : I.sig_face[0], I.g, H0, Q0, H1,
                         Q1, c00, c01, c11, Hg0, Qg0, Hg1, Qg1);
        if (p0 == 1) { H[0] = Hg0; Q[0] = Qg0; }
        else { H[1] = Hg0; Q[1] = Qg0; H[0] = Hg1; Q[0] = Qg1; }
    }
    if (j > N - 3) {
        const int pb = N - 1 - j + 2;  // position of cell N-1 (2 or 3)
        double Hg0, Qg0, Hg1, Qg1;
        double H0 = pb == 3 ? H[3] : H[2], Q0 = pb == 3 ? Q[3] : Q[2];
        double H1 = pb == 3 ? H[2] : H[1], Q1 = pb == 3 ? Q[2] : Q[1];
        const double c00 = SURF ? I.z_avg[N + 1] - I.z_avg[N + 2] : 0.0;
        const double c01 = SURF ? I.z_avg[N + 1] - I.z_avg[N + 3] : 0.0;
        const double c11 = SURF ? I.z_avg[N] - I.z_avg[N + 3] : 0.0;
        ghost_pair<SURF>(I.bc_kind[1], I.bc_q[1], I.bc_h[1], SURF ? 1.0 : I.sig_face[N], I.g, H0, Q0, H1,
                         Q1, c00, c01, c11, Hg0, Qg0, Hg1, Qg1);
        if (pb == 3) { H[4] = Hg0; Q[4] = Qg0; }
        else { H[3] = Hg0; Q[3] = Qg0; H[4] = Hg1; Q[4] = Qg1; }
    }
}

// Source of eq. (9) from the four face values of H feeding the cubic U_h.  SURF: the four face
// values are of the surface eta, eta_j = H_j + zbar_j, and -g int h b_x over the cell is split
// exactly into -g [int (eta_h - eta_j) b_x + eta_j (b_{j+1/2} - b_{j-1/2}) - (b_{j+1/2}^2 -
// b_{j-1/2}^2) / 2], the integral by the same two-point Gauss rule; a still surface then gives
// R = 0 to rounding on any bottom.
template <bool SURF>
__device__ __forceinline__ double source_term(double Hp_ll, double Hp_l, double Hm_r, double Hm_rr,
                                              const CellGeom &G, const CubicGauss &W, double dx,
                                              double g, double eta_j)
{
    if (SURF) {
        double quad = 0.0;
#pragma unroll
        for (int q = 0; q < 2; q++) {
            const double eg = W.w[q][0] * Hp_ll + W.w[q][1] * Hp_l + W.w[q][2] * Hm_r + W.w[q][3] * Hm_rr;
            quad = quad + (eg - eta_j) * G.bxg[q];
        }
        return -g * (0.5 * dx * quad + eta_j * (G.zfp - G.zfm) - 0.5 * (G.zfp * G.zfp - G.zfm * G.zfm));
    }
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < 2; q++) {
        double Hg = W.w[q][0] * Hp_ll + W.w[q][1] * Hp_l + W.w[q][2] * Hm_r + W.w[q][3] * Hm_rr;
        double hg = Hg * G.isg[q];
        double s = 0.5 * g * hg * hg * G.sxg[q] - g * G.sg[q] * hg * G.bxg[q];
        sum = sum + s;
    }
    return 0.5 * dx * sum;
}

// The reconstructions a local residual needs (section 3.1, Figure 1b): for each component the
// two states at x_{j-1/2} and at x_{j+1/2}; for H also the outer nodes of the source cubic.
struct Recon {
    double Hm_l, Hp_l, Hm_r, Hp_r, Hp_ll, Hm_rr;
    double Qm_l, Qp_l, Qm_r, Qp_r;
};

__device__ __forceinline__ void recon_H(const double H[5], Recon &r)
{
    r.Hm_l = weno_minus(H[0], H[1], H[2]);   // U-_{j-1/2}, from cell j-1
    r.Hp_l = weno_plus(H[1], H[2], H[3]);    // U+_{j-1/2}, from cell j
    r.Hm_r = weno_minus(H[1], H[2], H[3]);   // U-_{j+1/2}, from cell j
    r.Hp_r = weno_plus(H[2], H[3], H[4]);    // U+_{j+1/2}, from cell j+1
    r.Hp_ll = weno_plus(H[0], H[1], H[2]);   // U+_{j-3/2}, from cell j-1
    r.Hm_rr = weno_minus(H[2], H[3], H[4]);  // U-_{j+3/2}, from cell j+1
}

__device__ __forceinline__ void recon_Q(const double Q[5], Recon &r)
{
    r.Qm_l = weno_minus(Q[0], Q[1], Q[2]);
    r.Qp_l = weno_plus(Q[1], Q[2], Q[3]);
    r.Qm_r = weno_minus(Q[1], Q[2], Q[3]);
    r.Qp_r = weno_plus(Q[2], Q[3], Q[4]);
}

// R_j = F(U-_{j+1/2}, U+_{j+1/2}) - F(U-_{j-1/2}, U+_{j-1/2}) - S_j  (eq. 10)
// SURF: the reconstructed H values are surface values; the depths are eta - b at the face
template <bool SURF>
__device__ __forceinline__ void assemble_residual(const Recon &r, double S, const CellGeom &G,
                                                  double g, double &R0, double &R1)
{
    double Fm0, Fm1, Fp0, Fp1;
    if (SURF) {
        hll(r.Hm_l - G.zfm, r.Qm_l, r.Hp_l - G.zfm, r.Qp_l, 1.0, 1.0, g, Fm0, Fm1);
        hll(r.Hm_r - G.zfp, r.Qm_r, r.Hp_r - G.zfp, r.Qp_r, 1.0, 1.0, g, Fp0, Fp1);
    } else {
        hll(r.Hm_l, r.Qm_l, r.Hp_l, r.Qp_l, G.sfm, G.isfm, g, Fm0, Fm1);
        hll(r.Hm_r, r.Qm_r, r.Hp_r, r.Qp_r, G.sfp, G.isfp, g, Fp0, Fp1);
    }
    R0 = Fp0 - Fm0;
    R1 = Fp1 - Fm1 - S;
}

// Local residual of eq. (10) from a ghost-complete stencil.
// SURF: H holds the surface H + zbar of the five cells
template <bool SURF>
__device__ __forceinline__ void local_residual(const double H[5], const double Q[5],
                                               const CellGeom &G, const CubicGauss &W,
                                               double dx, double g, double &R0, double &R1)
{
    Recon r;
    recon_H(H, r);
    recon_Q(Q, r);
    const double S = source_term<SURF>(r.Hp_ll, r.Hp_l, r.Hm_r, r.Hm_rr, G, W, dx, g, H[2]);
    assemble_residual<SURF>(r, S, G, g, R0, R1);
}

// Stage U[a-2 .. a+kTile+1] of one instance into LDS (zeros outside the grid).
template <bool STREAM = false>
__device__ __forceinline__ void stage_state(const Inst1D &I, int a, double (*sH), double (*sQ))
{
    for (int k = threadIdx.x; k < kTile + 4; k += kTile) {
        int c = a - 2 + k;
        bool ok = c >= 0 && c < I.N;
        sH[k] = ok ? ldg<STREAM>(&I.U[c]) : 0.0;
        sQ[k] = ok ? ldg<STREAM>(&I.U[I.N + c]) : 0.0;
    }
}

__device__ __forceinline__ bool inst_active(const NewtonState *state, const Inst1D &I)
{
    return state == nullptr || state[I.active_idx].active;
}

__device__ double block_sum(double v, double *scratch)
{
    // wavefront reduction then a fixed-order sum over the 4 wavefronts
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kTile / 64; w++) s += scratch[w];
    return s;
}

// the surface H + zbar of the five cells of a ghost-complete stencil
__device__ __forceinline__ void to_surface(double H[5], const Inst1D &I, int j)
{
#pragma unroll
    for (int p = 0; p < 5; p++) H[p] = H[p] + I.z_avg[j + p];
}

template <bool SURF>
__device__ void residual_tile(const Inst1D &I, int a, double *partial_out)
{
    __shared__ double sH[kTile + 4], sQ[kTile + 4];
    __shared__ double red[kTile / 64];
    stage_state(I, a, sH, sQ);
    __syncthreads();
    const int j = a + threadIdx.x;
    double n1 = 0.0;
    if (j < I.N) {
        double H[5], Q[5];
#pragma unroll
        for (int p = 0; p < 5; p++) { H[p] = sH[threadIdx.x + p]; Q[p] = sQ[threadIdx.x + p]; }
        stencil_ghosts<SURF>(H, Q, j, I);
        if (SURF) to_surface(H, I, j);
        CellGeom G = load_geom<SURF>(I, j);
        CubicGauss W;
        double R0, R1;
        local_residual<SURF>(H, Q, G, W, I.dx, I.g, R0, R1);
        I.R[j] = R0;
        I.R[I.N + j] = R1;
        n1 = fabs(R0) + fabs(R1);
        I.rn[j] = n1;
    }
    double s = block_sum(n1, red);
    if (threadIdx.x == 0 && partial_out) *partial_out = s;
}

template <bool SURF>
__global__ void __launch_bounds__(kTile) k_residual_batch(const Inst1D *insts, const Tile *tiles,
                                                          NewtonState *state, double *partial)
{
    const Tile t = tiles[blockIdx.x];
    const Inst1D &I = insts[t.lev];
    if (!inst_active(state, I)) return;
    residual_tile<SURF>(I, t.a, partial + blockIdx.x);
}

template <bool SURF>
__global__ void __launch_bounds__(kTile) k_residual_single(Inst1D I)
{
    residual_tile<SURF>(I, blockIdx.x * kTile, nullptr);
}

// res = (1/N) sum_j rn_j for a single instance: one workgroup, fixed order.
__global__ void __launch_bounds__(kTile) k_sum_res(const double *rn, int N, double *res)
{
    __shared__ double red[kTile / 64];
    double v = 0.0;
    for (int j = threadIdx.x; j < N; j += kTile) v += rn[j];
    double s = block_sum(v, red);
    if (threadIdx.x == 0) *res = s / N;
}

// Per instance (one wavefront each): res from the tile partials (fixed order: lane-strided
// sums, then a fixed shuffle tree), the Newton counter and the stopping test of Algorithm 1
// (res < tol or n >= n_max; a non-finite res stops the instance with an error).
__global__ void __launch_bounds__(64) k_res_finalize(const Inst1D *insts, int ninst, NewtonState *state,
                                                     const double *partial, int init)
{
    const int b = blockIdx.x;
    if (b >= ninst) return;
    const Inst1D &I = insts[b];
    NewtonState &S = state[I.active_idx];
    if (!init && !S.active) return;
    double v = 0.0;
    for (int k = threadIdx.x; k < I.res_tiles; k += 64) v += partial[I.res_tile0 + k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (threadIdx.x != 0) return;
    const double res = v / I.N;
    S.res = res;
    S.sor_done = 0;   // the next Newton step starts a fresh inner iteration
    if (init) {
        S.n = I.n_start;
        S.active = 1;
        S.status = NMG_NOT_CONVERGED;
        if (!(res == res) || res > 1e300) { S.active = 0; S.status = NMG_ENONFINITE; }
        return;
    }
    if (I.hist && S.n < I.max_hist) I.hist[S.n] = res;
    S.n += 1;
    if (!(res == res) || res > 1e300) { S.active = 0; S.status = NMG_ENONFINITE; }
    else if (res < I.tol) { S.active = 0; S.status = NMG_OK; }
    else if (S.n >= I.n_max) { S.active = 0; S.status = NMG_NOT_CONVERGED; }
}

// ---- Jacobian --------------------------------------------------------------------------
// Column (i, m) of eq. (12) perturbs component m of cell i; the kernel evaluates the local
// residual of each row for each column of its stencil.
//
// Away from the boundaries (no ghost moves with a perturbation) the rows share their faces: the
// face k+1/2 between cells k and k+1 reads the four cells k-1..k+2 (its left state is cell k's
// minus reconstruction over k-1..k+1, its right state cell k+1's plus reconstruction over
// k..k+2), and the rows of cells k and k+1 both need its flux for the unperturbed state and for
// a perturbation of any of those cells (a column of either row), with identical operands.  So
// one lane evaluates one face, for the unperturbed state and each of the eight perturbations
// (four cells, two components), and each row is assembled from its two faces' fluxes and, for
// the source of eq. (9), the H states of four faces, taken from the neighbouring lanes.  Every
// flux, state and source is formed from the same operands by the same operations as when a row
// re-evaluates its own stencil, so the rows are those of the per-row evaluation bit for bit,
// with 9 instead of 14 flux evaluations and 16 instead of 40 reconstructions per row (J3).

// Fluxes and H states of one face k+1/2.
struct FaceVals {
    double fb0, fb1;     // flux, unperturbed
    double fh[4][2];     // flux with H of cell k-1+o perturbed, o = 0..3
    double fq[4][2];     // flux with Q of cell k-1+o perturbed
    double hl[4];        // left H state: unperturbed, then with cell k-1+o perturbed (index 1+o, o = 0..2)
    double hr[4];        // right H state: unperturbed, then with cell k-1+o perturbed (index o, o = 1..3)
};

// cells k-1..k+2 of face k+1/2 from the staged tile (cells a-2 .. a+kTile+1; zeros beyond);
// SURF: surface values H + zbar.  CHECK = false: the caller's faces lie inside the staged cells
// (a lane's own face, k = a + threadIdx.x - 1, reads staged cells threadIdx.x .. threadIdx.x + 3)
template <bool SURF, bool CHECK = true>
__device__ __forceinline__ void face_stencil(const Inst1D &I, const double *sH, const double *sQ, int a, int k,
                                             double h[4], double q[4])
{
#pragma unroll
    for (int p = 0; p < 4; p++) {
        const int st = k - 1 + p - (a - 2);
        const bool in = !CHECK || (st >= 0 && st < kTile + 4);
        h[p] = in ? sH[st] : 0.0;
        q[p] = in ? sQ[st] : 0.0;
        if (SURF) {
            const int z = k + 1 + p;   // z_avg holds cells -2..N+1 at index cell + 2
            h[p] = h[p] + ((z >= 0 && z <= I.N + 3) ? I.z_avg[z] : 0.0);
        }
    }
}

// width (and its reciprocal) or bottom of face k+1/2 (face k+1 of the face arrays)
template <bool SURF>
__device__ __forceinline__ void face_geom(const Inst1D &I, int k, double &sig, double &isig, double &zf)
{
    const int f = k + 1;
    const bool in = f >= 0 && f <= I.N;
    if (SURF) {
        sig = isig = 1.0;
        zf = in ? I.z_face[f] : 0.0;
    } else {
        sig = in ? I.sig_face[f] : 1.0;
        isig = qrcp(sig);
        zf = 0.0;
    }
}

template <bool SURF>
__device__ __forceinline__ void face_flux(double hl, double ql, double hr, double qr, double sig, double isig,
                                          double zf, double g, double &f0, double &f1)
{
    if (SURF) hll(hl - zf, ql, hr - zf, qr, 1.0, 1.0, g, f0, f1);
    else hll(hl, ql, hr, qr, sig, isig, g, f0, f1);
}

template <bool SURF>
__device__ __forceinline__ void face_eval(const double h[4], const double q[4], double sig, double isig, double zf,
                                          double eps, double g, FaceVals &F)
{
    const double HL = weno_minus(h[0], h[1], h[2]), HR = weno_plus(h[1], h[2], h[3]);
    const double QL = weno_minus(q[0], q[1], q[2]), QR = weno_plus(q[1], q[2], q[3]);
    face_flux<SURF>(HL, QL, HR, QR, sig, isig, zf, g, F.fb0, F.fb1);
    F.hl[0] = HL;
    F.hr[0] = HR;
#pragma unroll
    for (int o = 0; o < 4; o++) {
        double x[4];
#pragma unroll
        for (int p = 0; p < 4; p++) x[p] = p == o ? h[p] + eps : h[p];
        const double hl = o <= 2 ? weno_minus(x[0], x[1], x[2]) : HL;
        const double hr = o >= 1 ? weno_plus(x[1], x[2], x[3]) : HR;
        if (o <= 2) F.hl[1 + o] = hl;
        if (o >= 1) F.hr[o] = hr;
        face_flux<SURF>(hl, QL, hr, QR, sig, isig, zf, g, F.fh[o][0], F.fh[o][1]);
    }
#pragma unroll
    for (int o = 0; o < 4; o++) {
        double y[4];
#pragma unroll
        for (int p = 0; p < 4; p++) y[p] = p == o ? q[p] + eps : q[p];
        const double ql = o <= 2 ? weno_minus(y[0], y[1], y[2]) : QL;
        const double qr = o >= 1 ? weno_plus(y[1], y[2], y[3]) : QR;
        face_flux<SURF>(HL, ql, HR, qr, sig, isig, zf, g, F.fq[o][0], F.fq[o][1]);
    }
}

// Faces a tile needs beyond one per lane: the right face of its last cell (k = a+255, all nine
// states), the left H states of face a+256 and the right H states of face a-2 (the outer nodes of
// the first and last cells' source cubics).  Item 0..8: face a+255 unperturbed, H of cell k-1+o
// perturbed (items 1..4), Q perturbed (5..8); items 9..12: left H state of face a+256,
// unperturbed then o = 0..2; items 13..16: right H state of face a-2, unperturbed then o = 1..3.
// Every item runs the same operations (four reconstructions and one flux), each lane one item.
constexpr int kFaceExtras = 17;

template <bool SURF>
__device__ __forceinline__ void face_extra(const Inst1D &I, const double *sH, const double *sQ, int a, int item,
                                           double eps, FaceVals &last, double *hl_after, double *hr_before)
{
    int k, oh = -1, oq = -1;
    if (item <= 8) {
        k = a + kTile - 1;
        if (item >= 1 && item <= 4) oh = item - 1;
        else if (item >= 5) oq = item - 5;
    } else if (item <= 12) {
        k = a + kTile;
        if (item >= 10) oh = item - 10;
    } else {
        k = a - 2;
        if (item >= 14) oh = item - 13;
    }
    double h[4], q[4], x[4], y[4];
    face_stencil<SURF>(I, sH, sQ, a, k, h, q);
#pragma unroll
    for (int p = 0; p < 4; p++) {
        x[p] = p == oh ? h[p] + eps : h[p];
        y[p] = p == oq ? q[p] + eps : q[p];
    }
    const double HL = weno_minus(x[0], x[1], x[2]), HR = weno_plus(x[1], x[2], x[3]);
    const double QL = weno_minus(y[0], y[1], y[2]), QR = weno_plus(y[1], y[2], y[3]);
    double sig, isig, zf, f0, f1;
    face_geom<SURF>(I, k, sig, isig, zf);
    face_flux<SURF>(HL, QL, HR, QR, sig, isig, zf, I.g, f0, f1);
    if (item == 0) {
        last.fb0 = f0; last.fb1 = f1; last.hl[0] = HL; last.hr[0] = HR;
    } else if (item <= 4) {
        last.fh[oh][0] = f0; last.fh[oh][1] = f1;
        if (oh <= 2) last.hl[1 + oh] = HL;
        if (oh >= 1) last.hr[oh] = HR;
    } else if (item <= 8) {
        last.fq[oq][0] = f0; last.fq[oq][1] = f1;
    } else if (item <= 12) {
        hl_after[item - 9] = HL;
    } else {
        hr_before[item - 13] = HR;
    }
}

// a wavefront-wide shift of v by one lane with a DPP move on each 32-bit half: CTRL 0x130 gives
// every lane the value of lane + 1, 0x138 that of lane - 1 (the lane past the end receives 0)
template <int CTRL>
__device__ __forceinline__ double wave_shift(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// the same shift with the lane past the end keeping `edge` instead (a DPP move whose source lane
// does not exist leaves its destination as it was)
template <int CTRL>
__device__ __forceinline__ double wave_shift_or(double v, double edge)
{
    const long long b = __double_as_longlong(v), e = __double_as_longlong(edge);
    const int lo = __builtin_amdgcn_update_dpp((int)e, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(e >> 32), (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// the value v of lane + 1 of the wavefront (its last lane: `edge`, the next face kept in LDS)
__device__ __forceinline__ double from_right(double v, double edge)
{
    return wave_shift_or<0x130>(v, edge);
}

// the value of lane + 2 (lanes 62 and 63: the next two faces' values from LDS)
__device__ __forceinline__ double from_right2(double v, double edge1, double edge2)
{
    return wave_shift_or<0x130>(wave_shift_or<0x130>(v, edge1), edge2);
}

// the value of lane - 1 (lane 0: the previous face's value from LDS)
__device__ __forceinline__ double from_left(double v, double edge)
{
    return wave_shift_or<0x138>(v, edge);
}

__device__ __forceinline__ void inv2d(const double A[4], double B[4])
{
    double det = A[0] * A[3] - A[1] * A[2];
    B[0] = A[3] / det;
    B[1] = -A[1] / det;
    B[2] = -A[2] / det;
    B[3] = A[0] / det;
}

// Rows of cells 2jc, 2jc+1 (fine blocks b = 0..nb-1) -> coarse tridiagonal row (eq. 17),
// summed in the order of child row, then child column.
template <int NB>
__device__ __forceinline__ void coarse_from_children(const double *f0, const double *f1,
                                                     double Wc[4], double Dc[4], double Ec[4])
{
#pragma unroll
    for (int e = 0; e < 4; e++) {
        if (NB == 5) {
            Wc[e] = f0[0 * 4 + e] + f0[1 * 4 + e] + f1[0 * 4 + e];
            Dc[e] = f0[2 * 4 + e] + f0[3 * 4 + e] + f1[1 * 4 + e] + f1[2 * 4 + e];
            Ec[e] = f0[4 * 4 + e] + f1[3 * 4 + e] + f1[4 * 4 + e];
        } else {
            Wc[e] = f0[0 * 4 + e];
            Dc[e] = f0[1 * 4 + e] + f0[2 * 4 + e] + f1[0 * 4 + e] + f1[1 * 4 + e];
            Ec[e] = f1[2 * 4 + e];
        }
    }
}

// v of the lane d places up in the same row of 16 lanes (DPP row shift; d = 1, 2, 4 or 8)
__device__ __forceinline__ double row_shift_down(double v, int d)
{
    switch (d) {
    case 1: return wave_shift<0x101>(v);
    case 2: return wave_shift<0x102>(v);
    case 4: return wave_shift<0x104>(v);
    default: return wave_shift<0x108>(v);
    }
}

// one coarse row (W, D, E blocks) into the level's operator [3][2][2][n] at cell jc
template <typename T>
__device__ __forceinline__ void put_coarse_row(const double r[12], T *Jc, int n, int jc, bool lead)
{
    if (lead && jc < n) {
#pragma unroll
        for (int e = 0; e < 12; e++) __builtin_nontemporal_store((T)r[e], &Jc[e * (long long)n + jc]);
    }
}

// Jacobian rows of one tile.  With `mg` levels (batched path) the tile also writes the finest
// right-hand side and the coarse operators of all levels that lie inside the tile (up to
// eight: 256 -> 1 cells).  FUSED: the tile evaluates the residual R_j of its rows itself (the
// base of every difference quotient, and the finest right-hand side), with the same operations
// as the residual kernel, instead of reading R and ||R_j||_1; it writes the tile's sum of
// ||R_j||_1 to *partial_out for the stopping test (every thread of the workgroup calls this).
template <typename T, int NB, bool SURF, bool FUSED = false>
__device__ void jacobian_tile(const Inst1D &I, int a, T *J, int stride, T *rhs,
                              const MGArgs *mg, const Level1D *L0, double *partial_out = nullptr)
{
    __shared__ double sH[kTile + 4], sQ[kTile + 4];
    __shared__ double rows[kTile * NB * 4];
    __shared__ double red[kTile / 64];
    __shared__ FaceVals next_face[kTile / 64];       // the face after each wavefront's last face
    __shared__ double next_hl2[kTile / 64][4];       // left H states of the face after that
    __shared__ double prev_hr[kTile / 64][4];        // right H states of the face before the first
    stage_state<true>(I, a, sH, sQ);   // the state, geometry and residual: last use this step
    // the coarse levels inside the tile (up to eight below the finest; an instance's levels are
    // consecutive in the level table, level l holding N / 2^l cells): their sizes and operator
    // offsets
    const int nlev = (mg && !L0->coarsest) ? (I.levels - 1 < 8 ? I.levels - 1 : 8) : 0;
    int lev_n[8];
    long long lev_J[8];
#pragma unroll
    for (int i = 0; i < 8; i++) {
        lev_n[i] = I.N >> (i + 1);
        lev_J[i] = i < nlev ? mg->levs[I.lev0 + 1 + i].J : 0;
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int j = a + t;
    const int lane = t & 63, wv = t >> 6;
    constexpr int HW = NB / 2;
    double *myrow = &rows[t * NB * 4];   // this cell's block row, in LDS
#pragma unroll
    for (int e = 0; e < NB * 4; e++) myrow[e] = 0.0;
    const double eps = I.eps, ieps = 1.0 / I.eps;

    // every lane evaluates the face to the left of its cell (k = j - 1); the extra faces of the
    // tile go to the lanes of the last wavefront
    FaceVals F;
    double h2;   // H (SURF: surface) of this lane's cell
    {
        double h[4], q[4], sig, isig, zf;
        face_stencil<SURF, false>(I, sH, sQ, a, j - 1, h, q);
        face_geom<SURF>(I, j - 1, sig, isig, zf);
        face_eval<SURF>(h, q, sig, isig, zf, eps, I.g, F);
        h2 = h[2];
    }
    if (wv >= 1 && lane == 0) next_face[wv - 1] = F;
    if (wv >= 1 && lane == 1) {
#pragma unroll
        for (int e = 0; e < 4; e++) next_hl2[wv - 1][e] = F.hl[e];
    }
    if (wv + 1 < kTile / 64 && lane == 63) {
#pragma unroll
        for (int e = 0; e < 4; e++) prev_hr[wv + 1][e] = F.hr[e];
    }
    if (wv == kTile / 64 - 1 && lane < kFaceExtras)
        face_extra<SURF>(I, sH, sQ, a, lane, eps, next_face[kTile / 64 - 1], next_hl2[kTile / 64 - 1], prev_hr[0]);
    __syncthreads();

    const bool valid = j < I.N;
    const bool interior = j >= 2 && j <= I.N - 3;
    const CellGeom G = load_geom<SURF, true>(I, valid ? j : I.N - 1);
    const CubicGauss W;
    double R0 = 0.0, R1 = 0.0, rn = 0.0;
    if (!FUSED && valid) {
        R0 = ldg<true>(&I.R[j]);
        R1 = ldg<true>(&I.R[I.N + j]);
        rn = ldg<true>(&I.rn[j]);
    }
    double n1 = 0.0;   // ||R_j||_1 of this row (FUSED)

    // rows of the interior cells from the faces j-3/2 (lane - 1), j-1/2 (this lane), j+1/2
    // (lane + 1) and j+3/2 (lane + 2); every lane takes part in the exchanges
    {
        const FaceVals &E = next_face[wv];
        const double Pfb0 = from_right(F.fb0, E.fb0), Pfb1 = from_right(F.fb1, E.fb1);
        const double Phl0 = from_right(F.hl[0], E.hl[0]);
        const double PPhl0 = from_right2(F.hl[0], E.hl[0], next_hl2[wv][0]);
        const double LLhr0 = from_left(F.hr[0], prev_hr[wv][0]);
        const double S0 = source_term<SURF>(LLhr0, F.hr[0], Phl0, PPhl0, G, W, I.dx, I.g, h2);
        if (FUSED) {
            R0 = Pfb0 - F.fb0;
            R1 = Pfb1 - F.fb1 - S0;
            n1 = (valid && interior) ? fabs(R0) + fabs(R1) : 0.0;
            rn = n1;
        }
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const int d = b - HW;
            // column (j+d, H): the own face has cell j+d at o = d+2, the right face at o = d+1
            const double m0 = d + 2 <= 3 ? F.fh[d + 2 < 0 ? 0 : d + 2][0] : F.fb0;
            const double m1 = d + 2 <= 3 ? F.fh[d + 2 < 0 ? 0 : d + 2][1] : F.fb1;
            double p0 = Pfb0, p1 = Pfb1;
            if (d + 1 >= 0) {
                const int o = d + 1 > 3 ? 3 : d + 1;
                p0 = from_right(F.fh[o][0], E.fh[o][0]);
                p1 = from_right(F.fh[o][1], E.fh[o][1]);
            }
            // the source's four face states with cell j+d perturbed
            const double sll = (d + 3 >= 1 && d + 3 <= 3) ? from_left(F.hr[d + 3 < 1 ? 1 : (d + 3 > 3 ? 3 : d + 3)],
                                                                      prev_hr[wv][d + 3 < 1 ? 1 : (d + 3 > 3 ? 3 : d + 3)])
                                                          : LLhr0;
            const double spl = (d + 2 >= 1 && d + 2 <= 3) ? F.hr[d + 2 < 1 ? 1 : (d + 2 > 3 ? 3 : d + 2)] : F.hr[0];
            const double smr = (d + 2 >= 1 && d + 2 <= 3) ? from_right(F.hl[d + 2 < 1 ? 1 : (d + 2 > 3 ? 3 : d + 2)],
                                                                       E.hl[d + 2 < 1 ? 1 : (d + 2 > 3 ? 3 : d + 2)])
                                                          : Phl0;
            const double smrr = (d + 1 >= 1 && d + 1 <= 3)
                                    ? from_right2(F.hl[d + 1 < 1 ? 1 : (d + 1 > 3 ? 3 : d + 1)],
                                                  E.hl[d + 1 < 1 ? 1 : (d + 1 > 3 ? 3 : d + 1)],
                                                  next_hl2[wv][d + 1 < 1 ? 1 : (d + 1 > 3 ? 3 : d + 1)])
                                    : PPhl0;
            const double S = source_term<SURF>(sll, spl, smr, smrr, G, W, I.dx, I.g, d == 0 ? h2 + eps : h2);
            const double P0 = p0 - m0, P1 = p1 - m1 - S;
            double e0 = (P0 - R0) * ieps, e1 = (P1 - R1) * ieps;
            if (d == 0) e0 += I.alpha * rn;
            if (valid && interior) {
                myrow[(b * 2 + 0) * 2 + 0] = e0;
                myrow[(b * 2 + 1) * 2 + 0] = e1;
            }
        }
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const int d = b - HW;
            const double m0 = d + 2 <= 3 ? F.fq[d + 2 < 0 ? 0 : d + 2][0] : F.fb0;
            const double m1 = d + 2 <= 3 ? F.fq[d + 2 < 0 ? 0 : d + 2][1] : F.fb1;
            double p0 = Pfb0, p1 = Pfb1;
            if (d + 1 >= 0) {
                const int o = d + 1 > 3 ? 3 : d + 1;
                p0 = from_right(F.fq[o][0], E.fq[o][0]);
                p1 = from_right(F.fq[o][1], E.fq[o][1]);
            }
            const double P0 = p0 - m0, P1 = p1 - m1 - S0;
            double e0 = (P0 - R0) * ieps, e1 = (P1 - R1) * ieps;
            if (d == 0) e1 += I.alpha * rn;
            if (valid && interior) {
                myrow[(b * 2 + 0) * 2 + 1] = e0;
                myrow[(b * 2 + 1) * 2 + 1] = e1;
            }
        }
    }
    if (valid) {
        if (!interior) {   // within two cells of a side: full re-evaluation with ghosts
            double H[5], Q[5];
#pragma unroll
            for (int p = 0; p < 5; p++) { H[p] = sH[t + p]; Q[p] = sQ[t + p]; }
            if (FUSED) {   // R from the ghost-complete unperturbed stencil
                double Hb[5], Qb[5];
#pragma unroll
                for (int p = 0; p < 5; p++) { Hb[p] = H[p]; Qb[p] = Q[p]; }
                stencil_ghosts<SURF>(Hb, Qb, j, I);
                if (SURF) to_surface(Hb, I, j);
                local_residual<SURF>(Hb, Qb, G, W, I.dx, I.g, R0, R1);
                n1 = fabs(R0) + fabs(R1);
                rn = n1;
            }
#pragma unroll 1
            for (int b = 0; b < NB; b++) {
                const int i = j + b - HW;
                const bool col_ok = i >= 0 && i < I.N;
                const int pp = 2 + b - HW;  // stencil position of the perturbed cell
#pragma unroll 1
                for (int m = 0; m < 2; m++) {
                    double e0 = 0.0, e1 = 0.0;
                    if (col_ok) {
                        double Hp[5], Qp[5];
#pragma unroll
                        for (int p = 0; p < 5; p++) {
                            Hp[p] = (p == pp && m == 0) ? H[p] + eps : H[p];
                            Qp[p] = (p == pp && m == 1) ? Q[p] + eps : Q[p];
                        }
                        stencil_ghosts<SURF>(Hp, Qp, j, I);
                        if (SURF) to_surface(Hp, I, j);
                        double P0, P1;
                        local_residual<SURF>(Hp, Qp, G, W, I.dx, I.g, P0, P1);
                        e0 = (P0 - R0) * ieps;
                        e1 = (P1 - R1) * ieps;
                        if (b == HW) {
                            if (m == 0) e0 += I.alpha * rn;
                            else e1 += I.alpha * rn;
                        }
                    }
                    myrow[(b * 2 + 0) * 2 + m] = e0;
                    myrow[(b * 2 + 1) * 2 + m] = e1;
                }
            }
        }
        if (rhs) {   // the finest level's right-hand side of eq. (16) is R itself
            rhs[j] = (T)R0;
            rhs[stride + j] = (T)R1;
        }
#pragma unroll
        for (int e = 0; e < NB * 4; e++) J[e * (long long)stride + j] = (T)myrow[e];
    }
    if (FUSED) {
        const double sum = block_sum(n1, red);
        if (t == 0 && partial_out) *partial_out = sum;
    }
    if (!mg || L0->coarsest) return;

    // coarse operators of the levels inside this tile (eq. 17), stored with non-temporal hints:
    // they are read only after the finest level's first smoothing pass, which should find this
    // tile's fine rows, not these, in the memory-side cache.  Levels 1-5 in the first two
    // wavefronts: thread t forms coarse cell t of level 1 from two fine rows in LDS, and each
    // further level l pairs the lanes 2^(l-2) apart, the upper lane's row brought over by a DPP
    // row shift (the pairs stay within rows of 16 lanes); levels 6-8 in the first wavefront from
    // the eight level-5 rows, passed through LDS.
    __syncthreads();   // every fine row in LDS
    T *base_mg = reinterpret_cast<T *>(mg->mg);
    __shared__ double lev5[8 * 12];
    if (t < 128) {
        double r[12];
        coarse_from_children<NB>(&rows[(2 * t) * NB * 4], &rows[(2 * t + 1) * NB * 4], &r[0], &r[4], &r[8]);
        put_coarse_row(r, base_mg + lev_J[0], lev_n[0], (a >> 1) + t, true);
#pragma unroll
        for (int l = 1; l < 5; l++) {   // level l + 1
            if (l < nlev) {
                const int d = 1 << (l - 1);
                double p[12], q[12];
#pragma unroll
                for (int e = 0; e < 12; e++) p[e] = row_shift_down(r[e], d);
                coarse_from_children<3>(r, p, &q[0], &q[4], &q[8]);
#pragma unroll
                for (int e = 0; e < 12; e++) r[e] = q[e];
                put_coarse_row(r, base_mg + lev_J[l], lev_n[l], (a >> (l + 1)) + (t >> l), (t & (2 * d - 1)) == 0);
            }
        }
        if (nlev > 5 && (t & 15) == 0) {
#pragma unroll
            for (int e = 0; e < 12; e++) lev5[(t >> 4) * 12 + e] = r[e];
        }
    }
    if (nlev <= 5) return;
    __syncthreads();
    if (t >= 64) return;
    {
        const int c = t < 4 ? t : 3;
        double r[12];
        coarse_from_children<3>(&lev5[(2 * c) * 12], &lev5[(2 * c + 1) * 12], &r[0], &r[4], &r[8]);
        put_coarse_row(r, base_mg + lev_J[5], lev_n[5], (a >> 6) + t, t < 4);
#pragma unroll
        for (int l = 6; l < 8; l++) {   // levels 7 and 8
            if (l < nlev) {
                const int d = 1 << (l - 6);
                double p[12], q[12];
#pragma unroll
                for (int e = 0; e < 12; e++) p[e] = row_shift_down(r[e], d);
                coarse_from_children<3>(r, p, &q[0], &q[4], &q[8]);
#pragma unroll
                for (int e = 0; e < 12; e++) r[e] = q[e];
                put_coarse_row(r, base_mg + lev_J[l], lev_n[l], (a >> (l + 1)) + (t >> (l - 5)),
                               t < 4 && (t & (2 * d - 1)) == 0);
            }
        }
    }
}

// FUSED: the residual is evaluated in the same launch (partial: per-tile sums of ||R_j||_1 in
// the tile order of the residual's tile list); otherwise R and ||R_j||_1 are read.
template <typename T, int NB, bool SURF, bool FUSED>
__global__ void __launch_bounds__(kTile) k_jacobian_batch(MGArgs mg, const Tile *tiles, double *partial)
{
    // the last tiles first: the pass before this one streamed the same state and geometry in
    // tile order, so its last tiles' data are still in the memory-side cache
    const int ti = gridDim.x - 1 - blockIdx.x;
    const Tile t = tiles[ti];
    const Inst1D &I = mg.insts[t.lev];
    if (!inst_active(mg.state, I)) return;
    const Level1D L = mg.levs[I.lev0];
    if (L.nb != NB) return;
    T *base = reinterpret_cast<T *>(mg.mg);
    jacobian_tile<T, NB, SURF, FUSED>(I, t.a, base + L.J, L.n, base + L.rhs, &mg, &L, partial + ti);
}

template <int NB, bool SURF>
__global__ void __launch_bounds__(kTile) k_jacobian_single(Inst1D I, double *J)
{
    jacobian_tile<double, NB, SURF>(I, blockIdx.x * kTile, J, I.N, (double *)nullptr, (const MGArgs *)nullptr,
                              (const Level1D *)nullptr);
}

// ---- launchers ---------------------------------------------------------------------------

hipError_t launch_residual1d(const Inst1D *insts_dev, const Tile *tiles, int ntiles,
                             const Inst1D *single, NewtonState *state, double *partial, int recon,
                             hipStream_t s)
{
    const bool surf = recon == NMG_RECON_SURFACE;
    if (single) {
        int nt = (single->N + kTile - 1) / kTile;
        if (surf) hipLaunchKernelGGL(k_residual_single<true>, dim3(nt), dim3(kTile), 0, s, *single);
        else hipLaunchKernelGGL(k_residual_single<false>, dim3(nt), dim3(kTile), 0, s, *single);
    } else {
        if (ntiles == 0) return hipSuccess;
        if (surf)
            hipLaunchKernelGGL(k_residual_batch<true>, dim3(ntiles), dim3(kTile), 0, s, insts_dev, tiles, state,
                               partial);
        else
            hipLaunchKernelGGL(k_residual_batch<false>, dim3(ntiles), dim3(kTile), 0, s, insts_dev, tiles, state,
                               partial);
    }
    return hipGetLastError();
}

hipError_t launch_res_finalize(const Inst1D *insts_dev, int ninst, NewtonState *state,
                               const double *partial, int init, hipStream_t s)
{
    hipLaunchKernelGGL(k_res_finalize, dim3(ninst), dim3(64), 0, s, insts_dev, ninst, state,
                       partial, init);
    return hipGetLastError();
}

hipError_t launch_sum_res(const double *rn, int N, double *res, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_res, dim3(1), dim3(kTile), 0, s, rn, N, res);
    return hipGetLastError();
}

template <bool SURF, bool FUSED>
static void jacobian_batch_launches(const Tile *tiles, int ntiles, const MGArgs &mg, int prec, int nb_mask,
                                    double *partial, hipStream_t s)
{
    // one launch per stencil width present; each tile runs only the one its instance uses
    if (prec == NMG_FP32_MG) {
        if (nb_mask & 1)
            hipLaunchKernelGGL((k_jacobian_batch<float, 3, SURF, FUSED>), dim3(ntiles), dim3(kTile), 0, s, mg, tiles, partial);
        if (nb_mask & 2)
            hipLaunchKernelGGL((k_jacobian_batch<float, 5, SURF, FUSED>), dim3(ntiles), dim3(kTile), 0, s, mg, tiles, partial);
    } else {
        if (nb_mask & 1)
            hipLaunchKernelGGL((k_jacobian_batch<double, 3, SURF, FUSED>), dim3(ntiles), dim3(kTile), 0, s, mg, tiles, partial);
        if (nb_mask & 2)
            hipLaunchKernelGGL((k_jacobian_batch<double, 5, SURF, FUSED>), dim3(ntiles), dim3(kTile), 0, s, mg, tiles, partial);
    }
}

template <bool SURF>
static void jacobian_single_launch(const Inst1D *single, double *J_single, hipStream_t s)
{
    const int nt = (single->N + kTile - 1) / kTile;
    if (single->nb == 5)
        hipLaunchKernelGGL((k_jacobian_single<5, SURF>), dim3(nt), dim3(kTile), 0, s, *single, J_single);
    else
        hipLaunchKernelGGL((k_jacobian_single<3, SURF>), dim3(nt), dim3(kTile), 0, s, *single, J_single);
}

hipError_t launch_jacobian1d(const Inst1D *insts_dev, const Tile *tiles, int ntiles,
                             const Inst1D *single, double *J_single, const MGArgs &mg, int prec,
                             int nb_mask, int recon, hipStream_t s, double *fused_partial)
{
    (void)insts_dev;
    const bool surf = recon == NMG_RECON_SURFACE;
    if (single) {
        if (surf) jacobian_single_launch<true>(single, J_single, s);
        else jacobian_single_launch<false>(single, J_single, s);
        return hipGetLastError();
    }
    if (ntiles == 0) return hipSuccess;
    if (fused_partial) {
        if (surf) jacobian_batch_launches<true, true>(tiles, ntiles, mg, prec, nb_mask, fused_partial, s);
        else jacobian_batch_launches<false, true>(tiles, ntiles, mg, prec, nb_mask, fused_partial, s);
    } else {
        if (surf) jacobian_batch_launches<true, false>(tiles, ntiles, mg, prec, nb_mask, nullptr, s);
        else jacobian_batch_launches<false, false>(tiles, ntiles, mg, prec, nb_mask, nullptr, s);
    }
    return hipGetLastError();
}

}  // namespace nmg
