// libnmg host side for 2D problems (section 4): argument checks, workspace layout and the
// Newton driver of Algorithm 1 with the V-cycle of Algorithm 2 on the 2D hierarchy.
//
// Workspace layout (byte offsets, each 256-byte aligned):
//   state    : NewtonState
//   partial  : double[residual tiles]      (per-tile sums of ||R_ij||_1)
//   hist     : double[max_hist]
//   R, rn    : double [3][ny][nx], [ny][nx]
//   mg       : per level: J [nb*9][M_l], Dinv [9][M_l], rhs [3][M_l], dU [3][M_l] (nb = 9 or 21 on
//              the finest level, 5 below)
//              in double (NMG_FP64) or float (NMG_FP32_MG), cells in the level's colour-blocked
//              order (M_l slots, Perm2D); the caller's arrays stay in the natural order
//   lu       : LU factors and row permutation of the coarsest operator (double [M][M], int [M])
#include <algorithm>
#include <cstddef>
#include <cstring>
#include <string>
#include <vector>

#include "nmg_common.h"

namespace nmg {

namespace {

#define HIP_TRY2(expr)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return set_error(NMG_EHIP, (std::string(#expr) + ": " + hipGetErrorString(e_)).c_str()); \
    } while (0)

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

struct Plan2D {
    Inst2D I;
    int levels = 0, prec = NMG_FP64, nu1 = 0, nu2 = 0, nu3 = 1, n_max = 0, max_hist = 0, ntiles = 0;
    int check_every = 1;
    int sweeps = 0;            // smoother: the directional sweeps D1-D4 (NMG_LINEAR_MG_SWEEPS)
    int sched = 0;             // launch schedule (NMG_SCHED2D_* bits)
    int bottom_first = 0;      // first level of the one-workgroup bottom (launch_bottom2d)
    double tau = 0.0, omega = 1.0, tol = 0.0;
    std::vector<Level2D> L;
    size_t off_state = 0, off_partial = 0, off_hist = 0, off_R = 0, off_rn = 0, off_mg = 0, off_lu = 0, total = 0;
};

nmg_status check2d(const nmg_desc *d, const nmg_params *p, bool need_geometry = true)
{
    if (!d || !p) return set_error(NMG_EINVAL, "null desc or params");
    if (d->dim != 2) return set_error(NMG_EINVAL, "dim must be 2");
    if (d->nx < 1 || d->ny < 1) return set_error(NMG_EINVAL, "nx and ny must be positive");
    if (d->levels < 1 || d->levels > kMaxLevels) return set_error(NMG_EINVAL, "levels must be in [1, 16]");
    const int f = 1 << (d->levels - 1);
    if (d->nx % f != 0 || d->ny % f != 0)
        return set_error(NMG_EINVAL, "nx and ny must be divisible by 2^(levels-1)");
    if ((long long)(d->nx / f) * (d->ny / f) > kMaxCoarse2D)
        return set_error(NMG_EINVAL, "coarsest 2D level has more than 40 cells; add levels");
    if ((long long)d->nx * d->ny > (1LL << 28)) return set_error(NMG_EINVAL, "grid too large");
    if (d->jac != 9 && d->jac != 21) return set_error(NMG_EINVAL, "2D jac must be 9 or 21");
    if (d->recon != NMG_RECON_CONSERVED && d->recon != NMG_RECON_SURFACE)
        return set_error(NMG_EINVAL, "recon must be NMG_RECON_CONSERVED or NMG_RECON_SURFACE");
    if (need_geometry && (!d->bx_gp || !d->by_gp)) return set_error(NMG_EINVAL, "null geometry pointer");
    if (need_geometry && d->recon == NMG_RECON_SURFACE && (!d->z_face || !d->z_avg))
        return set_error(NMG_EINVAL, "recon = NMG_RECON_SURFACE needs z_face and z_avg");
    if (!(d->x1 > d->x0) || !(d->y1 > d->y0)) return set_error(NMG_EINVAL, "empty domain");
    for (int k = 0; k < 4; k++)
        if (d->bc[k].kind < NMG_BC_DISCHARGE || d->bc[k].kind > NMG_BC_STATE)
            return set_error(NMG_EINVAL, "bad boundary kind");
    if (!(p->eps > 0.0)) return set_error(NMG_EINVAL, "eps must be positive");
    if (p->nu1 < 0 || p->nu2 < 0 || p->nu3 < 1 || p->n_max < 0)
        return set_error(NMG_EINVAL, "bad nu1/nu2/nu3/n_max");
    if (p->nu1 > 1000 || p->nu2 > 1000 || p->nu3 > 1000) return set_error(NMG_EINVAL, "nu above 1000");
    if (p->precision != NMG_FP64 && p->precision != NMG_FP32_MG) return set_error(NMG_EINVAL, "bad precision");
    if (p->linear != NMG_LINEAR_MG && p->linear != NMG_LINEAR_MG_SWEEPS)
        return set_error(NMG_EINVAL, "2D linear must be NMG_LINEAR_MG or NMG_LINEAR_MG_SWEEPS");
    if (p->linear == NMG_LINEAR_MG_SWEEPS && (long long)d->nx * d->ny > 65536)
        return set_error(NMG_EINVAL, "the directional sweeps take grids of at most 65536 cells");
    if (p->schedule < 0 || p->schedule >= NMG_TUNE2D_CANDIDATES) return set_error(NMG_EINVAL, "bad 2D schedule");
    return NMG_OK;
}

Inst2D make_inst2d(const nmg_desc *d, const nmg_params *p)
{
    Inst2D I;
    memset(&I, 0, sizeof(I));
    I.Nx = d->nx;
    I.Ny = d->ny;
    I.dx = (d->x1 - d->x0) / d->nx;
    I.dy = (d->y1 - d->y0) / d->ny;
    I.g = d->g;
    I.x0 = d->x0;
    I.y0 = d->y0;
    for (int k = 0; k < 4; k++) {
        I.bc_kind[k] = d->bc[k].kind;
        I.bc_q[k] = d->bc[k].q;
        I.bc_h[k] = d->bc[k].h;
        I.bc_u[k] = d->bc[k].u;
        I.bc_v[k] = d->bc[k].v;
    }
    I.wall_x = d->wall_x;
    I.bx = d->bx_gp;
    I.by = d->by_gp;
    I.recon = d->recon;
    if (d->recon == NMG_RECON_SURFACE) {
        I.zavg = d->z_avg;
        I.zfx = d->z_face;
        I.zfy = d->z_face ? d->z_face + (long long)d->ny * (d->nx + 1) * 2 : nullptr;
    }
    I.alpha = p ? p->alpha : 0.0;
    I.eps = p ? p->eps : 1.0;
    return I;
}

// the first level of the one-workgroup bottom: the levels of at most kBottom2DCells cells (128
// with NMG_SCHED2D_SMALL_BOTTOM) down to the coarsest
void set_bottom(Plan2D &P)
{
    const long long lim = (P.sched & NMG_SCHED2D_SMALL_BOTTOM) ? 128 : kBottom2DCells;
    P.bottom_first = P.levels - 1;
    while (P.bottom_first > 0 && (long long)P.L[P.bottom_first - 1].nx * P.L[P.bottom_first - 1].ny <= lim)
        P.bottom_first--;
}

nmg_status build2d(Plan2D &P, const nmg_desc *d, const nmg_params *p, bool need_geometry = true)
{
    nmg_status st = check2d(d, p, need_geometry);
    if (st != NMG_OK) return st;
    P.I = make_inst2d(d, p);
    P.levels = d->levels;
    P.prec = p->precision;
    P.nu1 = p->nu1;
    P.nu2 = p->nu2;
    P.nu3 = p->nu3;
    P.n_max = p->n_max;
    P.max_hist = std::min(std::max(p->n_max, 1), 100000);
    P.check_every = std::max(1, p->check_every);
    P.sweeps = p->linear == NMG_LINEAR_MG_SWEEPS ? 1 : 0;
    P.sched = p->schedule;
    P.tau = p->tau;
    P.omega = p->omega;
    P.tol = p->tol;
    P.ntiles = residual2d_tiles(d->nx, d->ny);
    const size_t vsz = P.prec == NMG_FP32_MG ? 4 : 8;
    long long e = 0;
    P.L.clear();
    for (int l = 0; l < P.levels; l++) {
        Level2D L;
        memset(&L, 0, sizeof(L));
        L.nx = d->nx >> l;
        L.ny = d->ny >> l;
        L.nb = l == 0 ? d->jac : 5;
        // colours of the cross (3), the full stencil (9) or the five-point stencil (2)
        L.P = make_perm2d(L.nx, L.ny, l == 0 ? (d->jac == 21 ? 9 : 3) : 2);
        const long long n = L.P.M;
        L.J = e; e += (long long)L.nb * 9 * n;
        L.Dinv = e; e += 9 * n;
        L.rhs = e; e += 3 * n;
        L.dU = e; e += 3 * n;
        e = (e + 63) & ~63LL;
        P.L.push_back(L);
    }
    const long long n0 = (long long)d->nx * d->ny;
    size_t o = 0;
    P.off_state = o; o = al256(o + sizeof(NewtonState));
    P.off_partial = o; o = al256(o + sizeof(double) * P.ntiles);
    P.off_hist = o; o = al256(o + sizeof(double) * P.max_hist);
    P.off_R = o; o = al256(o + sizeof(double) * 3 * n0);
    P.off_rn = o; o = al256(o + sizeof(double) * n0);
    P.off_mg = o; o = al256(o + vsz * (size_t)e);
    const Level2D &Lc = P.L.back();
    set_bottom(P);
    P.off_lu = o; o = al256(o + coarse_lu_bytes(3 * Lc.nx * Lc.ny));
    P.total = o;
    return NMG_OK;
}

// nu smoothing iterations on level l, each two symmetric multicolour steps (colours 0..C-1, then
// C-1..0).  Consecutive passes of one colour (C-1 C-1 at a turn, 0 0 between steps) see the same
// neighbour values and run as one launch that relaxes twice.
nmg_status smooth(const Plan2D &P, char *mgb, int l, int nu, hipStream_t s)
{
    const Level2D &L = P.L[l];
    if (P.sweeps) {
        if (nu > 0) HIP_TRY2(launch_sweeps2d(mgb, L, nu, P.omega, P.prec, s));
        return NMG_OK;
    }
    const int C = L.P.C;
    int cur = -1, run = 0;
    for (int it = 0; it < nu; it++)
        for (int half = 0; half < 4; half++)
            for (int q = 0; q < C; q++) {
                const int c = (half & 1) ? C - 1 - q : q;
                if (c == cur) { run++; continue; }
                if (run > 0) HIP_TRY2(launch_smooth2d_pass(mgb, L, cur, run, P.omega, P.prec, s, P.sched));
                cur = c;
                run = 1;
            }
    if (run > 0) HIP_TRY2(launch_smooth2d_pass(mgb, L, cur, run, P.omega, P.prec, s, P.sched));
    return NMG_OK;
}

// Algorithm 2 from level l (recursive)
nmg_status vcycle_from(const Plan2D &P, char *mgb, int l, hipStream_t s)
{
    if (l >= P.bottom_first) {
        HIP_TRY2(launch_bottom2d(mgb, P.L.data(), l, P.levels, P.nu1, P.nu2, P.omega,
                                 (const double *)(mgb - P.off_mg + P.off_lu), P.prec, s, P.sweeps));
        return NMG_OK;
    }
    nmg_status st;
    if ((st = smooth(P, mgb, l, P.nu1, s)) != NMG_OK) return st;
    HIP_TRY2(launch_restrict2d(mgb, P.L[l], P.L[l + 1], P.prec, s));
    if ((st = vcycle_from(P, mgb, l + 1, s)) != NMG_OK) return st;
    HIP_TRY2(launch_prolong2d(mgb, P.L[l], P.L[l + 1], P.prec, s));
    return smooth(P, mgb, l, P.nu2, s);
}

// coarse operators of every level below the finest, then the factors of the coarsest
nmg_status coarsen_all(const Plan2D &P, char *mgb, hipStream_t s)
{
    for (int l = 1; l < P.levels; l++) HIP_TRY2(launch_coarsen2d(mgb, P.L[l - 1], P.L[l], P.prec, s));
    HIP_TRY2(launch_coarse_factor2d(mgb, P.L.back(), (double *)(mgb - P.off_mg + P.off_lu), P.prec, s));
    return NMG_OK;
}

Inst2D bound_inst(const Plan2D &P, char *w, double *U)
{
    Inst2D I = P.I;
    I.U = U;
    I.R = (double *)(w + P.off_R);
    I.rn = (double *)(w + P.off_rn);
    return I;
}

// one Newton step of Algorithm 1 (all device work, no host synchronisation)
nmg_status newton_step(const Plan2D &P, char *w, double *U, hipStream_t s)
{
    const Inst2D I = bound_inst(P, w, U);
    char *mgb = w + P.off_mg;
    const size_t vsz = P.prec == NMG_FP32_MG ? 4 : 8;
    const Level2D &L0 = P.L[0];
    const long long n0 = (long long)L0.nx * L0.ny;
    NewtonState *S = (NewtonState *)(w + P.off_state);
    HIP_TRY2(launch_jacobian2d(I, L0.P, mgb + vsz * L0.J, mgb + vsz * L0.rhs, mgb + vsz * L0.Dinv, P.prec, s, L0.nb));
    nmg_status st = coarsen_all(P, mgb, s);
    if (st != NMG_OK) return st;
    HIP_TRY2(launch_fill(mgb + vsz * L0.dU, P.prec, 3 * L0.P.M, s));
    for (int m = 0; m < P.nu3; m++)
        if ((st = vcycle_from(P, mgb, 0, s)) != NMG_OK) return st;
    HIP_TRY2(launch_update2d(U, mgb, L0, P.tau, S, P.prec, s));
    HIP_TRY2(launch_residual2d(I, (double *)(w + P.off_partial), s));
    HIP_TRY2(launch_state2d((double *)(w + P.off_partial), P.ntiles, n0, P.tol, P.n_max, S,
                            (double *)(w + P.off_hist), P.max_hist, 0, s));
    return NMG_OK;
}

}  // namespace

size_t workspace2d_bytes(const nmg_desc *d, const nmg_params *p)
{
    Plan2D P;
    if (build2d(P, d, p, false) != NMG_OK) return 0;
    return P.total;
}

nmg_status residual2d(const nmg_desc *d, const double *U, double *R, double *rn, double *res, hipStream_t s)
{
    nmg_params p;
    memset(&p, 0, sizeof(p));
    p.eps = 1.0;
    p.nu3 = 1;
    nmg_status st = check2d(d, &p);
    if (st != NMG_OK) return st;
    if (!U || !R || !rn) return set_error(NMG_EINVAL, "null U/R/rn");
    Inst2D I = make_inst2d(d, &p);
    I.U = const_cast<double *>(U);
    I.R = R;
    I.rn = rn;
    HIP_TRY2(launch_residual2d(I, nullptr, s));
    if (res) HIP_TRY2(launch_sum_res(rn, d->nx * d->ny, res, s));
    return NMG_OK;
}

nmg_status jacobian2d(const nmg_desc *d, const nmg_params *p, const double *U, const double *R,
                      const double *rn, double *J, hipStream_t s)
{
    nmg_status st = check2d(d, p);
    if (st != NMG_OK) return st;
    if (!U || !R || !rn || !J) return set_error(NMG_EINVAL, "null U/R/rn/J");
    Inst2D I = make_inst2d(d, p);
    I.U = const_cast<double *>(U);
    I.R = const_cast<double *>(R);
    I.rn = const_cast<double *>(rn);
    HIP_TRY2(launch_jacobian2d(I, make_perm2d(d->nx, d->ny, 1), J, nullptr, nullptr, NMG_FP64, s, d->jac));
    return NMG_OK;
}

nmg_status vcycle2d(const nmg_desc *d, const nmg_params *p, void *ws, size_t ws_bytes, const void *J,
                    const void *rhs, void *dU, int setup, hipStream_t s)
{
    if (!ws || !rhs || !dU || (setup && !J)) return set_error(NMG_EINVAL, "null argument");
    Plan2D P;
    nmg_status st = build2d(P, d, p);
    if (st != NMG_OK) return st;
    if (ws_bytes < P.total) return set_error(NMG_ENOMEM_WS, "workspace too small");
    char *mgb = (char *)ws + P.off_mg;
    const size_t vsz = P.prec == NMG_FP32_MG ? 4 : 8;
    const Level2D &L0 = P.L[0];
    if (setup) {
        HIP_TRY2(launch_permute2d(J, NMG_FP64, mgb + vsz * L0.J, P.prec, L0, 9 * L0.nb, 1, s));
        HIP_TRY2(launch_dinv2d((const double *)J, mgb + vsz * L0.Dinv, L0, P.prec, s));
        if ((st = coarsen_all(P, mgb, s)) != NMG_OK) return st;
    }
    HIP_TRY2(launch_permute2d(rhs, P.prec, mgb + vsz * L0.rhs, P.prec, L0, 3, 1, s));
    HIP_TRY2(launch_permute2d(dU, P.prec, mgb + vsz * L0.dU, P.prec, L0, 3, 1, s));
    if ((st = vcycle_from(P, mgb, 0, s)) != NMG_OK) return st;
    HIP_TRY2(launch_permute2d(mgb + vsz * L0.dU, P.prec, dU, P.prec, L0, 3, 0, s));
    return NMG_OK;
}

// Stepwise form of the Newton driver: begin evaluates the residual of U and initialises the
// state in the workspace; steps enqueues `steps` Newton steps and an asynchronous copy of the
// state to the host.  Neither waits for the device.
static_assert(sizeof(NewtonState) == sizeof(nmg_newton_state), "nmg_newton_state mirrors the device state");
static_assert(offsetof(NewtonState, n) == offsetof(nmg_newton_state, iters) &&
                  offsetof(NewtonState, active) == offsetof(nmg_newton_state, active) &&
                  offsetof(NewtonState, status) == offsetof(nmg_newton_state, status),
              "nmg_newton_state mirrors the device state");

nmg_status newton2d_begin(const nmg_desc *d, const nmg_params *p, void *ws, size_t ws_bytes, double *U, hipStream_t s)
{
    if (!ws || !U) return set_error(NMG_EINVAL, "null argument");
    Plan2D P;
    nmg_status st = build2d(P, d, p);
    if (st != NMG_OK) return st;
    if (ws_bytes < P.total) return set_error(NMG_ENOMEM_WS, "workspace too small");
    char *w = (char *)ws;
    const Inst2D I = bound_inst(P, w, U);
    const long long n0 = (long long)P.L[0].nx * P.L[0].ny;
    HIP_TRY2(launch_residual2d(I, (double *)(w + P.off_partial), s));
    HIP_TRY2(launch_state2d((double *)(w + P.off_partial), P.ntiles, n0, P.tol, P.n_max,
                            (NewtonState *)(w + P.off_state), nullptr, 0, 1, s));
    return NMG_OK;
}

nmg_status newton2d_steps(const nmg_desc *d, const nmg_params *p, void *ws, size_t ws_bytes, double *U, int steps,
                          nmg_newton_state *state_out, hipStream_t s)
{
    if (!ws || !U) return set_error(NMG_EINVAL, "null argument");
    if (steps < 0) return set_error(NMG_EINVAL, "steps must be >= 0");
    Plan2D P;
    nmg_status st = build2d(P, d, p);
    if (st != NMG_OK) return st;
    if (ws_bytes < P.total) return set_error(NMG_ENOMEM_WS, "workspace too small");
    char *w = (char *)ws;
    for (int k = 0; k < steps; k++)
        if ((st = newton_step(P, w, U, s)) != NMG_OK) return st;
    if (state_out)
        HIP_TRY2(hipMemcpyAsync(state_out, w + P.off_state, sizeof(NewtonState), hipMemcpyDeviceToHost, s));
    return NMG_OK;
}

nmg_status autotune2d(const nmg_desc *d, const nmg_params *p, void *ws, size_t ws_bytes, const double *J,
                      const void *rhs, int cycles, int *best, double *ms, hipStream_t s)
{
    if (!ws || !J || !rhs || !best || !ms) return set_error(NMG_EINVAL, "null argument");
    if (cycles < 1 || cycles > 1000) return set_error(NMG_EINVAL, "cycles must be in [1, 1000]");
    nmg_params q = *p;
    q.schedule = 0;
    Plan2D P;
    nmg_status st = build2d(P, d, &q);
    if (st != NMG_OK) return st;
    if (P.sweeps) return set_error(NMG_EINVAL, "the schedules concern the multicolour smoother");
    if (ws_bytes < P.total) return set_error(NMG_ENOMEM_WS, "workspace too small");
    char *mgb = (char *)ws + P.off_mg;
    const size_t vsz = P.prec == NMG_FP32_MG ? 4 : 8;
    const Level2D &L0 = P.L[0];
    HIP_TRY2(launch_permute2d(J, NMG_FP64, mgb + vsz * L0.J, P.prec, L0, 9 * L0.nb, 1, s));
    HIP_TRY2(launch_dinv2d(J, mgb + vsz * L0.Dinv, L0, P.prec, s));
    if ((st = coarsen_all(P, mgb, s)) != NMG_OK) return st;
    HIP_TRY2(launch_permute2d(rhs, P.prec, mgb + vsz * L0.rhs, P.prec, L0, 3, 1, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY2(hipEventCreate(&e0));
    struct Ev { hipEvent_t &a, &b; ~Ev() { if (a) (void)hipEventDestroy(a); if (b) (void)hipEventDestroy(b); } } guard{e0, e1};
    HIP_TRY2(hipEventCreate(&e1));
    int b = 0;
    for (int c = 0; c < NMG_TUNE2D_CANDIDATES; c++) {
        P.sched = c;
        set_bottom(P);
        HIP_TRY2(launch_fill(mgb + vsz * L0.dU, P.prec, 3 * L0.P.M, s));
        if ((st = vcycle_from(P, mgb, 0, s)) != NMG_OK) return st;          // warm-up
        HIP_TRY2(hipEventRecord(e0, s));
        for (int k = 0; k < cycles; k++)
            if ((st = vcycle_from(P, mgb, 0, s)) != NMG_OK) return st;
        HIP_TRY2(hipEventRecord(e1, s));
        HIP_TRY2(hipEventSynchronize(e1));
        float t = 0.0f;
        HIP_TRY2(hipEventElapsedTime(&t, e0, e1));
        ms[c] = t / cycles;
        if (ms[c] < ms[b]) b = c;
    }
    *best = b;
    return NMG_OK;
}

nmg_status newton2d(const nmg_desc *d, const nmg_params *p, void *ws, size_t ws_bytes, double *U,
                    nmg_stats *stats, double *hist, int max_hist, hipStream_t s)
{
    if (!ws || !U || !stats) return set_error(NMG_EINVAL, "null argument");
    Plan2D P;
    nmg_status st = build2d(P, d, p);
    if (st != NMG_OK) return st;
    if (ws_bytes < P.total) return set_error(NMG_ENOMEM_WS, "workspace too small");
    char *w = (char *)ws;
    const Inst2D I = bound_inst(P, w, U);
    const long long n0 = (long long)P.L[0].nx * P.L[0].ny;
    NewtonState *S = (NewtonState *)(w + P.off_state);
    HIP_TRY2(launch_residual2d(I, (double *)(w + P.off_partial), s));
    HIP_TRY2(launch_state2d((double *)(w + P.off_partial), P.ntiles, n0, P.tol, P.n_max, S, nullptr, 0, 1, s));
    NewtonState hs;
    memset(&hs, 0, sizeof(hs));
    HIP_TRY2(hipMemcpyAsync(&hs, S, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIP_TRY2(hipStreamSynchronize(s));
    // Steps are enqueued check_every at a time; once the device state stops, the remaining
    // enqueued steps leave U unchanged (the update kernel reads the state).
    while (hs.active) {
        for (int k = 0; k < P.check_every; k++)
            if ((st = newton_step(P, w, U, s)) != NMG_OK) return st;
        HIP_TRY2(hipMemcpyAsync(&hs, S, sizeof(hs), hipMemcpyDeviceToHost, s));
        HIP_TRY2(hipStreamSynchronize(s));
    }
    stats->iters = hs.n;
    stats->status = hs.status;
    stats->res = hs.res;
    if (hist && max_hist > 0) {
        const int cnt = std::min(std::min(max_hist, hs.n), P.max_hist);
        if (cnt > 0) {
            HIP_TRY2(hipMemcpyAsync(hist, w + P.off_hist, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
            HIP_TRY2(hipStreamSynchronize(s));
        }
    }
    return (nmg_status)hs.status;
}

}  // namespace nmg
