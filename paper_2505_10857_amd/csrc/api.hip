// libnmg host side: argument checking, workspace layout, the Newton driver of Algorithm 1 and
// the batched plan.  All device work is launched from here onto the caller's stream.
//
// Workspace layout (byte offsets, each 256-byte aligned):
//   tables   : Inst1D[n] | Level1D[nlev] | Tile[...] | int inst_list[n]
//   state    : NewtonState[n]
//   partial  : double[res tiles]            (per-tile sums of ||R_j||_1)
//   hist     : double[n][max_hist]
//   R, rn    : double, per instance [2N] and [N]
//   mg       : per instance and level: J [nb*4][n_l], rhs [2][n_l], dU [2][n_l]
//              in double (NMG_FP64) or float (NMG_FP32_MG)
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "nmg_common.h"

using namespace nmg;

namespace {

thread_local std::string g_err;

nmg_status fail(nmg_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(NMG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));        \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

nmg_status check_desc1d(const nmg_desc *d, const nmg_params *p, bool need_geometry = true)
{
    if (!d || !p) return fail(NMG_EINVAL, "null desc or params");
    if (d->dim != 1) return fail(NMG_EINVAL, "only dim = 1 is handled by this entry point");
    if (d->nx < 4) return fail(NMG_EINVAL, "nx must be >= 4");
    if (p->linear != NMG_LINEAR_MG && p->linear != NMG_LINEAR_SOR && p->linear != NMG_LINEAR_SOR_LEX)
        return fail(NMG_EINVAL, "bad linear solver");
    if (p->linear != NMG_LINEAR_MG) {   // Newton-SOR: no hierarchy
        if (p->sor_max < 1 || p->sor_max > 1000) return fail(NMG_EINVAL, "sor_max must be in [1, 1000]");
        if (!(p->sor_tol >= 0.0)) return fail(NMG_EINVAL, "sor_tol must be >= 0");
    } else {
        if (d->levels < 1 || d->levels > kMaxLevels) return fail(NMG_EINVAL, "levels must be in [1, 16]");
        if (d->levels == 1 && d->jac != 3)
            return fail(NMG_EINVAL, "a one-level hierarchy (direct solve) needs the three-block Jacobian");
        if (d->nx % (1 << (d->levels - 1)) != 0)
            return fail(NMG_EINVAL, "nx must be divisible by 2^(levels-1)");
        if ((d->nx >> (d->levels - 1)) > kMaxCoarse)
            return fail(NMG_EINVAL, "coarsest level has more than 256 cells; add levels");
    }
    if (d->jac != 3 && d->jac != 5) return fail(NMG_EINVAL, "1D jac must be 3 or 5");
    if (d->recon != NMG_RECON_CONSERVED && d->recon != NMG_RECON_SURFACE)
        return fail(NMG_EINVAL, "bad recon");
    if (need_geometry && (!d->sig_face || !d->sig_gp || !d->sigx_gp || !d->bx_gp))
        return fail(NMG_EINVAL, "null geometry pointer");
    if (need_geometry && d->recon == NMG_RECON_SURFACE && (!d->z_face || !d->z_avg))
        return fail(NMG_EINVAL, "the surface reconstruction needs z_face and z_avg");
    if (!(d->x1 > d->x0)) return fail(NMG_EINVAL, "x1 must exceed x0");
    if (!(p->eps > 0.0)) return fail(NMG_EINVAL, "eps must be positive");
    if (p->nu1 < 0 || p->nu2 < 0 || p->nu3 < 1 || p->n_max < 0)
        return fail(NMG_EINVAL, "bad nu1/nu2/nu3/n_max");
    if (p->nu1 > 8 || p->nu2 > 8)
        return fail(NMG_EINVAL, "nu1/nu2 above 8 are not supported by the fused 1D smoother");
    if (p->precision != NMG_FP64 && p->precision != NMG_FP32_MG)
        return fail(NMG_EINVAL, "bad precision");
    return NMG_OK;
}

Inst1D make_inst(const nmg_desc *d, const nmg_params *p)
{
    Inst1D I;
    memset(&I, 0, sizeof(I));
    I.N = d->nx;
    I.levels = p->linear == NMG_LINEAR_MG ? d->levels : 1;   // Newton-SOR works on the grid alone
    I.nb = d->jac;
    I.dx = (d->x1 - d->x0) / d->nx;
    I.g = d->g;
    for (int s = 0; s < 2; s++) {
        I.bc_kind[s] = d->bc[s].kind;
        I.bc_q[s] = d->bc[s].q;
        I.bc_h[s] = d->bc[s].h;
    }
    I.sig_face = d->sig_face;
    I.sig_gp = d->sig_gp;
    I.sigx_gp = d->sigx_gp;
    I.bx_gp = d->bx_gp;
    I.recon = d->recon;
    I.z_face = d->z_face;
    I.z_avg = d->z_avg;
    I.alpha = p->alpha;
    I.tau = p->tau;
    I.eps = p->eps;
    I.omega = p->omega;
    I.tol = p->tol;
    I.nu1 = p->nu1;
    I.nu2 = p->nu2;
    I.nu3 = p->nu3;
    I.n_max = p->n_max;
    return I;
}

}  // namespace

nmg_status nmg::set_error(nmg_status st, const char *msg) { return fail(st, msg); }

// Pinned host blocks (a plan's staging of its instance table and its copy of the Newton states)
// are kept for reuse when a plan is destroyed instead of being freed: freeing pinned memory
// waits for the whole device, which would stall other streams' work every time a server
// re-plans.  The pool holds at most what the plans alive at one time used.
namespace {
std::mutex g_pin_mu;
std::multimap<size_t, void *> g_pin_free;          // size -> block
std::unordered_map<void *, size_t> g_pin_size;     // every block the pool made

hipError_t pinned_get(void **p, size_t bytes)
{
    bytes = (bytes + 4095) & ~size_t(4095);
    {
        std::lock_guard<std::mutex> lk(g_pin_mu);
        auto it = g_pin_free.lower_bound(bytes);
        if (it != g_pin_free.end() && it->first <= 4 * bytes) {
            *p = it->second;
            g_pin_free.erase(it);
            return hipSuccess;
        }
    }
    hipError_t e = hipHostMalloc(p, bytes);
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_pin_mu);
        g_pin_size[*p] = bytes;
    }
    return e;
}

void pinned_put(void *p)
{
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_pin_mu);
    auto it = g_pin_size.find(p);
    if (it != g_pin_size.end()) g_pin_free.insert({it->second, p});
}
}  // namespace

struct nmg_plan {
    int n = 0;
    int prec = NMG_FP64;
    int nu3 = 1;
    int check_every = 1;
    std::vector<Inst1D> insts;
    std::vector<Level1D> levs;
    std::vector<Tile> tiles;                  // all tile lists, concatenated
    int res_t0 = 0, res_nt = 0;               // residual / Jacobian tiles
    std::vector<std::pair<int, int>> coarsen; // (t0, nt) per coarsening pass from level 0
    std::vector<std::pair<int, int>> coarsen8;// (t0, nt) per pass from level 8 (Newton path)
    std::vector<std::pair<int, int>> smooth;  // (t0, nt) per depth
    std::vector<int> smooth_mask;             // stencil widths present per depth (bit0: 3, bit1: 5)
    // finest-level tiles of the launch that runs one V-cycle's post-smoothing and the next one's
    // pre-smoothing (nu3 >= 2, every instance on three-block rows); count 0 when not used
    std::pair<int, int> fused0 = {0, 0};
    int jac_mask = 0;
    int depth = 0;
    size_t off_insts = 0, off_levs = 0, off_tiles = 0, off_list = 0, off_state = 0, off_partial = 0,
           off_hist = 0, off_R = 0, off_mg = 0, total = 0;
    std::vector<size_t> R_off;                // per instance byte offset of R (rn follows)
    std::vector<int> n_start;                 // Newton steps already taken, per instance
    // tunables (nmg_plan_options) and what is needed to rebuild the tables for them
    int linear = NMG_LINEAR_MG;               // inner solver (nmg_params.linear)
    int sor_max = 0;
    double sor_tol = 0.0;
    int sor_t0 = 0, sor_nt = 0;               // Newton-SOR tiles (level 0, one-step halo)
    int bottom_cells = 2048;                  // levels up to this size run in k_bottom
    int recon = NMG_RECON_CONSERVED;          // reconstruction of every instance
    int bottom_nt = 1024;                     // its workgroup size
    int smooth_tile = kSmoothTile;            // cells per tile of the tiled multigrid smoother
    int split_finest = 0;                     // 1: no fused finest-level launch between cycles
    // 0: the residual is evaluated inside the Jacobian launch at the end of each Newton step
    // (the next step's Jacobian), 1: a separate residual launch ends each step and the Jacobian
    // starts the next
    int split_residual = 0;
    size_t tile_cap = 0;                      // tile-table entries reserved (any option fits)
    std::vector<nmg_desc> descs;
    std::vector<nmg_params> params;
    int max_hist = 0;
    // graph cache
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    void *g_ws = nullptr;
    hipStream_t own_stream = nullptr;
    hipEvent_t order_ev = nullptr;            // orders own_stream after the caller's null-stream work
    NewtonState *host_state = nullptr;        // pinned
    char *host_tables = nullptr;              // pinned staging of the instance table
    bool host_borrowed = false;               // host_state / host_tables belong to the caller
    void *tables_ws = nullptr;                // workspace whose static tables are current
    // kernel timing
    int prof_kernel = NMG_K_NONE;
    std::vector<hipEvent_t> ev_pool;          // created lazily, reused
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_open;
    hipStream_t prof_stream = nullptr;
    double prof_ms = 0.0;
    int prof_count = 0;
    ~nmg_plan()
    {
        for (auto e : ev_pool) (void)hipEventDestroy(e);
        for (auto &pr : ev_open) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (own_stream) (void)hipStreamDestroy(own_stream);
        if (order_ev) (void)hipEventDestroy(order_ev);
        if (!host_borrowed) {
            pinned_put(host_state);
            pinned_put(host_tables);
        }
    }
};

namespace {

nmg_status build_plan(nmg_plan *P, const nmg_desc *descs, const nmg_params *params, int n,
                      bool need_geometry = true)
{
    if (n <= 0) return fail(NMG_EINVAL, "need at least one instance");
    P->n = n;
    P->prec = params[0].precision;
    P->nu3 = params[0].nu3;
    P->check_every = std::max(1, params[0].check_every);
    P->linear = params[0].linear;
    P->sor_max = params[0].sor_max;
    P->sor_tol = params[0].sor_tol;
    P->recon = descs[0].recon;
    for (int k = 0; k < n; k++) {
        nmg_status st = check_desc1d(&descs[k], &params[k], need_geometry);
        if (st != NMG_OK) return fail(st, "instance " + std::to_string(k) + ": " + g_err);
        if (params[k].precision != P->prec) return fail(NMG_EINVAL, "mixed precisions in one plan");
        if (params[k].nu3 != P->nu3) return fail(NMG_EINVAL, "mixed nu3 in one plan");
        if (params[k].linear != P->linear || params[k].sor_max != P->sor_max || !(params[k].sor_tol == P->sor_tol))
            return fail(NMG_EINVAL, "mixed linear solvers in one plan");
        if (descs[k].recon != P->recon) return fail(NMG_EINVAL, "mixed reconstructions in one plan");
    }
    const size_t vsz = P->prec == NMG_FP32_MG ? sizeof(float) : sizeof(double);
    P->insts.clear();
    P->levs.clear();
    P->tiles.clear();
    int max_levels = 0;
    P->max_hist = 0;
    for (int k = 0; k < n; k++) {
        max_levels = std::max(max_levels, P->linear == NMG_LINEAR_MG ? descs[k].levels : 1);
        P->max_hist = std::max(P->max_hist, std::min(params[k].n_max, 100000));
    }
    P->depth = max_levels - 1;

    // levels and multigrid element offsets
    long long mg_elems = 0;
    std::vector<std::vector<int>> lev_index(n);
    for (int k = 0; k < n; k++) {
        Inst1D I = make_inst(&descs[k], &params[k]);
        I.active_idx = k;
        I.lev0 = (int)P->levs.size();
        for (int l = 0; l < I.levels; l++) {
            Level1D L;
            memset(&L, 0, sizeof(L));
            L.inst = k;
            L.l = l;
            L.n = I.N >> l;
            L.nb = l == 0 ? I.nb : 3;
            L.coarsest = l == I.levels - 1;
            L.halo = P->linear == NMG_LINEAR_MG ? smooth_halo(L.nb, std::max(I.nu1, I.nu2), 0)
                                                : halo_cells(L.nb, 1);
            L.V = (P->linear == NMG_LINEAR_MG ? P->smooth_tile : kTile) - 2 * L.halo;
            L.halo2 = smooth_halo(L.nb, I.nu2, I.nu1);
            L.V2 = P->smooth_tile - 2 * L.halo2;
            L.child = L.coarsest ? -1 : (int)P->levs.size() + 1;
            L.J = mg_elems; mg_elems += (long long)L.nb * 4 * L.n;
            L.rhs = mg_elems; mg_elems += 2LL * L.n;
            L.dU = mg_elems; mg_elems += 2LL * L.n;
            L.dUo = mg_elems; mg_elems += 2LL * L.n;
            L.aux = -1;
            if (P->linear == NMG_LINEAR_SOR_LEX && l == 0) { L.aux = mg_elems; mg_elems += 2LL * L.n; }
            mg_elems = (mg_elems + 63) & ~63LL;
            lev_index[k].push_back((int)P->levs.size());
            P->levs.push_back(L);
        }
        I.levc = (int)P->levs.size() - 1;
        // bottom kernel: from the first three-block level with at most bottom_cells cells
        I.lbot = I.levels - 1;
        for (int l = 0; l < I.levels; l++)
            if ((I.N >> l) <= P->bottom_cells && (l > 0 || I.nb == 3)) { I.lbot = l; break; }
        I.max_hist = std::min(params[k].n_max, 100000);
        P->insts.push_back(I);
    }
    // residual / Jacobian tiles
    P->res_t0 = 0;
    P->jac_mask = 0;
    for (int k = 0; k < n; k++) {
        P->insts[k].res_tile0 = (int)P->tiles.size();
        int nt = (P->insts[k].N + kTile - 1) / kTile;
        P->insts[k].res_tiles = nt;
        for (int t = 0; t < nt; t++) P->tiles.push_back({k, t * kTile});
        P->jac_mask |= P->insts[k].nb == 5 ? 2 : 1;
    }
    P->res_nt = (int)P->tiles.size();
    // Newton-SOR tiles: level 0 with the halo of one symmetric step
    P->sor_t0 = (int)P->tiles.size();
    if (P->linear == NMG_LINEAR_SOR) {
        for (int k = 0; k < n; k++) {
            const Level1D &L = P->levs[lev_index[k][0]];
            P->insts[k].sor_tile0 = (int)P->tiles.size() - P->sor_t0;
            for (int a = 0; a < L.n; a += L.V) P->tiles.push_back({lev_index[k][0], a});
            P->insts[k].sor_tiles = (int)P->tiles.size() - P->sor_t0 - P->insts[k].sor_tile0;
        }
    }
    P->sor_nt = (int)P->tiles.size() - P->sor_t0;
    // coarsening passes: each pass starts at level 10*p and builds up to ten more levels
    P->coarsen.clear();
    const int span = kTile * kCoarsenCells;
    for (int l0 = 0; l0 < max_levels; l0 += 10) {
        int t0 = (int)P->tiles.size();
        for (int k = 0; k < n; k++) {
            if (l0 >= P->insts[k].levels) continue;
            const Level1D &L = P->levs[lev_index[k][l0]];
            for (int a = 0; a < L.n; a += span) P->tiles.push_back({lev_index[k][l0], a});
        }
        P->coarsen.push_back({t0, (int)P->tiles.size() - t0});
    }
    // the Jacobian tiles (256 cells) build levels 1..8 themselves; deeper levels start at 8
    P->coarsen8.clear();
    for (int l0 = 8; l0 < max_levels - 1; l0 += 10) {
        int t0 = (int)P->tiles.size();
        for (int k = 0; k < n; k++) {
            if (l0 >= P->insts[k].levels - 1) continue;
            const Level1D &L = P->levs[lev_index[k][l0]];
            for (int a = 0; a < L.n; a += span) P->tiles.push_back({lev_index[k][l0], a});
        }
        P->coarsen8.push_back({t0, (int)P->tiles.size() - t0});
    }
    // smoothing tiles per depth
    P->smooth.clear();
    P->smooth_mask.clear();
    for (int d = 0; d < P->depth; d++) {
        int t0 = (int)P->tiles.size(), mask = 0;
        for (int k = 0; k < n; k++) {
            if (d >= P->insts[k].lbot) continue;
            const Level1D &L = P->levs[lev_index[k][d]];
            if (L.V < 2) return fail(NMG_EINVAL, "smoothing halo exceeds the tile");
            for (int a = 0; a < L.n; a += L.V) P->tiles.push_back({lev_index[k][d], a});
            mask |= L.nb == 5 ? 2 : 1;
        }
        P->smooth.push_back({t0, (int)P->tiles.size() - t0});
        P->smooth_mask.push_back(mask);
    }
    P->fused0 = {0, 0};
    if (P->linear == NMG_LINEAR_MG && P->nu3 >= 2 && P->jac_mask == 1 && P->depth > 0 && !P->split_finest) {
        bool ok = true;
        for (int k = 0; k < n && ok; k++)
            ok = P->levs[lev_index[k][0]].V2 >= P->smooth_tile / 2;   // at most twice the tiles
        if (ok) {
            int t0 = (int)P->tiles.size();
            for (int k = 0; k < n; k++) {
                if (P->insts[k].lbot == 0) continue;
                const Level1D &L = P->levs[lev_index[k][0]];
                for (int a = 0; a < L.n; a += L.V2) P->tiles.push_back({lev_index[k][0], a});
            }
            P->fused0 = {t0, (int)P->tiles.size() - t0};
        }
    }
    // byte layout
    size_t o = 0;
    P->off_insts = o; o = align256(o + sizeof(Inst1D) * n);
    P->off_levs = o; o = align256(o + sizeof(Level1D) * P->levs.size());
    P->off_tiles = o;
    o = align256(o + sizeof(Tile) * std::max<size_t>(1, std::max(P->tiles.size(), P->tile_cap)));
    P->off_list = o; o = align256(o + sizeof(int) * n);
    P->off_state = o; o = align256(o + sizeof(NewtonState) * n);
    P->off_partial = o; o = align256(o + sizeof(double) * std::max(1, std::max(P->res_nt, P->sor_nt)));
    P->off_hist = o; o = align256(o + sizeof(double) * (size_t)n * std::max(1, P->max_hist));
    P->R_off.resize(n);
    for (int k = 0; k < n; k++) {
        P->R_off[k] = o;
        o = align256(o + sizeof(double) * 3 * (size_t)P->insts[k].N);
    }
    P->off_mg = o; o = align256(o + vsz * (size_t)mg_elems);
    P->total = o;
    return NMG_OK;
}

hipEvent_t take_event(nmg_plan *P)
{
    if (!P->ev_pool.empty()) {
        hipEvent_t e = P->ev_pool.back();
        P->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Bracket one launch of kernel `k` with events when it is the profiled kernel.
struct ProfScope {
    nmg_plan *P;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(nmg_plan *P_, int k, hipStream_t s_, bool capturing) : P(P_), s(s_)
    {
        if (capturing || P->prof_kernel != k) return;
        a = take_event(P);
        b = take_event(P);
        if (a && b) (void)hipEventRecord(a, s);
    }
    ~ProfScope()
    {
        if (!a || !b) return;
        (void)hipEventRecord(b, s);
        P->ev_open.push_back({a, b});
        P->prof_stream = s;
    }
};

MGArgs mg_args(const nmg_plan *P, char *ws, bool with_state)
{
    MGArgs a;
    a.insts = reinterpret_cast<const Inst1D *>(ws + P->off_insts);
    a.levs = reinterpret_cast<const Level1D *>(ws + P->off_levs);
    a.state = with_state ? reinterpret_cast<NewtonState *>(ws + P->off_state) : nullptr;
    a.mg = ws + P->off_mg;
    return a;
}

// Upload the tables with the device pointers of this workspace and these states.  The level
// and tile tables depend only on the plan and the workspace and are uploaded once per
// workspace; the instance table (which holds the state pointers) is uploaded on every call,
// from pinned memory.
nmg_status upload_tables(nmg_plan *P, char *ws, double *const *U, hipStream_t s)
{
    if (P->tables_ws != ws) {
        std::vector<char> h(P->off_state - P->off_levs, 0);
        const size_t b = P->off_levs;
        memcpy(h.data() + P->off_levs - b, P->levs.data(), sizeof(Level1D) * P->levs.size());
        if (!P->tiles.empty())
            memcpy(h.data() + P->off_tiles - b, P->tiles.data(), sizeof(Tile) * P->tiles.size());
        std::vector<int> list(P->n);
        for (int k = 0; k < P->n; k++) list[k] = k;
        memcpy(h.data() + P->off_list - b, list.data(), sizeof(int) * P->n);
        HIP_TRY(hipMemcpyAsync(ws + b, h.data(), h.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        P->tables_ws = ws;
    }
    const size_t isz = sizeof(Inst1D) * P->n;
    if (!P->host_tables) HIP_TRY(pinned_get((void **)&P->host_tables, isz));
    else HIP_TRY(hipStreamSynchronize(s));   // the previous upload from this buffer has landed
    for (int k = 0; k < P->n; k++) {
        Inst1D I = P->insts[k];
        I.U = U ? U[k] : nullptr;
        I.R = reinterpret_cast<double *>(ws + P->R_off[k]);
        I.rn = I.R + 2 * (size_t)I.N;
        I.hist = reinterpret_cast<double *>(ws + P->off_hist) + (size_t)k * std::max(1, P->max_hist);
        I.n_start = P->n_start.empty() ? 0 : P->n_start[k];
        memcpy(P->host_tables + sizeof(Inst1D) * k, &I, sizeof(Inst1D));
    }
    HIP_TRY(hipMemcpyAsync(ws + P->off_insts, P->host_tables, isz, hipMemcpyHostToDevice, s));
    return NMG_OK;
}

const Tile *tiles_at(const nmg_plan *P, char *ws, int t0)
{
    return reinterpret_cast<const Tile *>(ws + P->off_tiles) + t0;
}

// Coarse operators of every level and their diagonal inverses.
nmg_status enqueue_setup(nmg_plan *P, char *ws, const MGArgs &mg, hipStream_t s, bool cap = true,
                         bool from_jacobian = false)
{
    for (auto &c : (from_jacobian ? P->coarsen8 : P->coarsen)) {
        ProfScope ps(P, NMG_K_COARSEN, s, cap);
        HIP_TRY(launch_coarsen1d(mg, tiles_at(P, ws, c.first), c.second, P->prec, s));
    }
    return NMG_OK;
}

// One V-cycle (Algorithm 2) over every instance.
// One V-cycle (Algorithm 2) over every instance.  Each tiled launch reads a level's dU from one
// of its two buffers and writes the other: below the finest level pre-smoothing writes dUo and
// post-smoothing reads it back into dU.  On the finest level `src0` names the buffer holding
// its current dU (0: dU, 1: dUo); `skip_pre0` leaves out its pre-smoothing (already done by the
// fused launch of the previous cycle) and `fuse_up0` replaces its post-smoothing by the fused
// launch that also pre-smooths for the next cycle.  Returns the finest level's buffer after the
// cycle in *src0_out.
nmg_status enqueue_vcycle(nmg_plan *P, char *ws, const MGArgs &mg, bool zero_init0, bool final_update,
                          hipStream_t s, bool cap = true, int src0 = 0, bool skip_pre0 = false,
                          bool fuse_up0 = false, int *src0_out = nullptr)
{
    const int *list = reinterpret_cast<const int *>(ws + P->off_list);
    for (int d = 0; d < P->depth; d++) {
        if (P->smooth[d].second == 0 || (d == 0 && skip_pre0)) continue;
        ProfScope ps(P, d == 0 ? NMG_K_SMOOTH_PRE : -1, s, cap);
        const int src = d == 0 ? src0 : 0;
        HIP_TRY(launch_smooth1d(mg, tiles_at(P, ws, P->smooth[d].first), P->smooth[d].second,
                                P->smooth_mask[d], 0, (d > 0 || zero_init0) ? 1 : 0, 0, src, P->prec, P->smooth_tile,
                                0, s));
        if (d == 0) src0 = 1 - src;
    }
    HIP_TRY(launch_bottom(mg, list, P->n, zero_init0 ? 1 : 0, final_update ? 1 : 0, P->prec, P->bottom_nt, s));
    // Passes alternate direction over data that a recent pass streamed, so that each begins in
    // the memory-side cache: the residual runs in tile order and the Jacobian after it in
    // reverse (k_jacobian_batch), so the finest pre-smoothing after that runs in order; a coarse
    // level's post-smoothing, with only smaller levels since its pre-smoothing, runs in reverse.
    for (int d = P->depth - 1; d >= 0; d--) {
        if (P->smooth[d].second == 0) continue;
        if (d == 0 && fuse_up0) {
            ProfScope ps(P, NMG_K_SMOOTH_FUSED, s, cap);
            HIP_TRY(launch_smooth1d(mg, tiles_at(P, ws, P->fused0.first), P->fused0.second, P->smooth_mask[0], 2,
                                    0, 0, src0, P->prec, P->smooth_tile, 0, s));
            src0 = 1 - src0;
            continue;
        }
        ProfScope ps(P, d == 0 ? NMG_K_SMOOTH_POST : -1, s, cap);
        const int src = d == 0 ? src0 : 1;
        HIP_TRY(launch_smooth1d(mg, tiles_at(P, ws, P->smooth[d].first), P->smooth[d].second,
                                P->smooth_mask[d], 1, 0, (d == 0 && final_update) ? 1 : 0, src, P->prec, P->smooth_tile,
                                d > 0 ? 1 : 0, s));
        if (d == 0) src0 = 1 - src;
    }
    if (src0_out) *src0_out = src0;
    return NMG_OK;
}

// One Newton step of Algorithm 1 for every active instance.  `cap`: being captured into a graph.
// The Jacobian of the current state and the residual norms behind the stopping test.  Fused
// (the default): one launch evaluates both (state: null while the Newton states are not yet
// initialised); split: the residual launch, then the Jacobian reads it.
nmg_status enqueue_residual_jacobian(nmg_plan *P, char *ws, const MGArgs &mg, hipStream_t s, bool cap)
{
    const Tile *rt = tiles_at(P, ws, P->res_t0);
    double *partial = reinterpret_cast<double *>(ws + P->off_partial);
    if (!P->split_residual) {
        ProfScope ps(P, NMG_K_JACOBIAN, s, cap);
        HIP_TRY(launch_jacobian1d(mg.insts, rt, P->res_nt, nullptr, nullptr, mg, P->prec, P->jac_mask, P->recon, s,
                                  partial));
        return NMG_OK;
    }
    {
        ProfScope ps(P, NMG_K_RESIDUAL, s, cap);
        HIP_TRY(launch_residual1d(mg.insts, rt, P->res_nt, nullptr, mg.state, partial, P->recon, s));
    }
    return NMG_OK;
}

nmg_status enqueue_split_jacobian(nmg_plan *P, char *ws, const MGArgs &mg, hipStream_t s, bool cap)
{
    ProfScope ps(P, NMG_K_JACOBIAN, s, cap);
    HIP_TRY(launch_jacobian1d(mg.insts, tiles_at(P, ws, P->res_t0), P->res_nt, nullptr, nullptr, mg, P->prec,
                              P->jac_mask, P->recon, s));
    return NMG_OK;
}

// One Newton step of Algorithm 1 for every active instance.  Fused order: the coarse operators
// beyond the Jacobian tile (the finest levels' were built with the Jacobian that ended the
// previous step), the linear solve and the damped update, then the next state's residual and
// Jacobian in one launch and the stopping test.  Split order: Jacobian, coarse operators, linear
// solve and update, residual, stopping test.  Both do the same arithmetic on the same values.
nmg_status enqueue_step(nmg_plan *P, char *ws, hipStream_t s, bool cap = false)
{
    MGArgs mg = mg_args(P, ws, true);
    const Inst1D *insts = mg.insts;
    const Tile *rt = tiles_at(P, ws, P->res_t0);
    NewtonState *state = mg.state;
    double *partial = reinterpret_cast<double *>(ws + P->off_partial);
    nmg_status st;
    if (P->split_residual && (st = enqueue_split_jacobian(P, ws, mg, s, cap)) != NMG_OK) return st;
    st = enqueue_setup(P, ws, mg, s, cap, true);
    if (st != NMG_OK) return st;
    if (P->linear == NMG_LINEAR_MG) {
        // with fused finest-level tiles, the post-smoothing of a cycle and the pre-smoothing of
        // the next run in one launch (nothing else touches the finest level between them)
        const bool fuse = P->fused0.second > 0;
        int src0 = 0;
        for (int v = 0; v < P->nu3; v++) {
            st = enqueue_vcycle(P, ws, mg, v == 0, v == P->nu3 - 1, s, cap, src0, fuse && v > 0,
                                fuse && v < P->nu3 - 1, &src0);
            if (st != NMG_OK) return st;
        }
    } else {
        // Newton-SOR: up to sor_max symmetric steps; an instance whose step changed dU by less
        // than sor_tol (l1) is skipped by the remaining ones
        const int nb_max = (P->jac_mask & 2) ? 5 : 3;
        for (int k = 0; k < P->sor_max; k++) {
            if (P->linear == NMG_LINEAR_SOR) {
                HIP_TRY(launch_sor_mc(mg, tiles_at(P, ws, P->sor_t0), P->sor_nt, nb_max, k, partial,
                                      P->prec, s));
                HIP_TRY(launch_sor_finalize(insts, P->n, state, partial, P->sor_tol, s));
            } else {
                HIP_TRY(launch_sor_lex(mg, P->n, nb_max, k == 0 ? 1 : 0, P->sor_tol, P->prec, s));
            }
        }
        // the multicolour steps alternate between the two dU buffers (the last one written is
        // dUo when the step count is odd); the lexicographic sweep works in dU
        const int from_out = P->linear == NMG_LINEAR_SOR && (P->sor_max & 1) ? 1 : 0;
        HIP_TRY(launch_update1d(mg, rt, P->res_nt, from_out, P->prec, s));
    }
    if ((st = enqueue_residual_jacobian(P, ws, mg, s, cap)) != NMG_OK) return st;
    HIP_TRY(launch_res_finalize(insts, P->n, state, partial, 0, s));
    return NMG_OK;
}

nmg_status plan_begin(nmg_plan *P, char *ws, size_t ws_bytes, double *const *U, hipStream_t s)
{
    if (!ws) return fail(NMG_EINVAL, "null workspace");
    if (ws_bytes < P->total) return fail(NMG_ENOMEM_WS, "workspace too small");
    if (!U) return fail(NMG_EINVAL, "null state array");
    for (int k = 0; k < P->n; k++)
        if (!U[k]) return fail(NMG_EINVAL, "null state pointer");
    nmg_status st = upload_tables(P, ws, U, s);
    if (st != NMG_OK) return st;
    if (P->g_ws != ws && P->gexec) {   // a graph captured on another workspace is stale
        (void)hipGraphExecDestroy(P->gexec);
        (void)hipGraphDestroy(P->graph);
        P->gexec = nullptr;
        P->graph = nullptr;
    }
    MGArgs mg = mg_args(P, ws, true);
    double *partial = reinterpret_cast<double *>(ws + P->off_partial);
    // the initial state's residual (and, fused, its Jacobian) for every instance: the Newton
    // states are initialised only by the stopping test that follows
    MGArgs all = mg;
    all.state = nullptr;
    nmg_status st2 = enqueue_residual_jacobian(P, ws, all, s, false);
    if (st2 != NMG_OK) return st2;
    HIP_TRY(launch_res_finalize(mg.insts, P->n, mg.state, partial, 1, s));
    return NMG_OK;
}

nmg_status read_state(nmg_plan *P, char *ws, hipStream_t s)
{
    if (!P->host_state) HIP_TRY(pinned_get((void **)&P->host_state, sizeof(NewtonState) * P->n));
    HIP_TRY(hipMemcpyAsync(P->host_state, ws + P->off_state, sizeof(NewtonState) * P->n,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return NMG_OK;
}

nmg_status plan_steps(nmg_plan *P, char *ws, int steps, int use_graph, hipStream_t s)
{
    if (use_graph) {
        if (!P->gexec || P->g_ws != ws) {
            hipStream_t cs = s;
            if (cs == nullptr) {   // the null stream cannot be captured: capture on the plan's own
                if (!P->own_stream) HIP_TRY(hipStreamCreateWithFlags(&P->own_stream, hipStreamNonBlocking));
                cs = P->own_stream;
            }
            HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            nmg_status st = enqueue_step(P, ws, cs, true);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(cs, &g);
            if (st != NMG_OK) { if (g) (void)hipGraphDestroy(g); return st; }
            if (e != hipSuccess) return fail(NMG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
            if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
            if (P->graph) (void)hipGraphDestroy(P->graph);
            P->graph = g;
            HIP_TRY(hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0));
            P->g_ws = ws;
        }
        hipStream_t ls = s ? s : P->own_stream;
        if (s == nullptr) {
            // after the caller's work on the null stream (an event, not a device-wide wait: work
            // of other streams, such as a server's 2D lane, goes on meanwhile)
            if (!P->order_ev) HIP_TRY(hipEventCreateWithFlags(&P->order_ev, hipEventDisableTiming));
            HIP_TRY(hipEventRecord(P->order_ev, nullptr));
            HIP_TRY(hipStreamWaitEvent(ls, P->order_ev, 0));
        }
        for (int k = 0; k < steps; k++) HIP_TRY(hipGraphLaunch(P->gexec, ls));
        if (s == nullptr) HIP_TRY(hipStreamSynchronize(ls));
        return NMG_OK;
    }
    for (int k = 0; k < steps; k++) {
        nmg_status st = enqueue_step(P, ws, s);
        if (st != NMG_OK) return st;
    }
    return NMG_OK;
}

constexpr int kBottomCandidates[4] = {256, 512, 1024, 2048};
constexpr int kTileCandidates[2] = {kSmoothTile, kSmoothTileMax};
static_assert(NMG_TUNE_CANDIDATES == 4 * 2 * 2 * 2,
              "tuner grid: bottom_cells x split_finest x smooth_tile x split_residual");

// Rebuild the plan's tables for another option set.  The byte layout does not move (the tile
// table is reserved for the largest tile count), so a workspace sized for the plan fits every
// option; device tables and any captured graph are refreshed on the next use.
nmg_status apply_options(nmg_plan *P, int cells, int split, int tile, int split_res)
{
    if (split_res != 0 && split_res != 1) return fail(NMG_EINVAL, "split_residual must be 0 or 1");
    bool ok = false;
    for (int c : kBottomCandidates) ok = ok || c == cells;
    if (!ok) return fail(NMG_EINVAL, "bottom_cells must be 256, 512, 1024 or 2048");
    if (tile == 0) tile = kSmoothTile;
    if (tile != kSmoothTile && tile != kSmoothTileMax) return fail(NMG_EINVAL, "smooth_tile must be 0, 256 or 512");
    if (split != 0 && split != 1) return fail(NMG_EINVAL, "split_finest must be 0 or 1");
    const size_t total = P->total;
    const int old_cells = P->bottom_cells, old_nt = P->bottom_nt, old_tile = P->smooth_tile, old_split = P->split_finest;
    P->bottom_cells = cells;
    P->bottom_nt = std::min(1024, std::max(256, cells / 2));
    P->smooth_tile = tile;
    P->split_finest = split;
    nmg_status st = build_plan(P, P->descs.data(), P->params.data(), P->n);
    if (st == NMG_OK && P->tiles.size() > P->tile_cap)
        st = fail(NMG_EINVAL, "option set needs more tiles than the plan reserved");
    if (st != NMG_OK) {   // keep the previous, valid tables
        const std::string err = g_err;
        P->bottom_cells = old_cells;
        P->bottom_nt = old_nt;
        P->smooth_tile = old_tile;
        P->split_finest = old_split;
        (void)build_plan(P, P->descs.data(), P->params.data(), P->n);
        P->total = std::max(P->total, total);
        return fail(st, err);
    }
    P->total = std::max(P->total, total);
    P->split_residual = split_res;
    P->tables_ws = nullptr;
    if (P->gexec) { (void)hipGraphExecDestroy(P->gexec); P->gexec = nullptr; }
    if (P->graph) { (void)hipGraphDestroy(P->graph); P->graph = nullptr; }
    return NMG_OK;
}

nmg_status plan_autotune(nmg_plan *P, char *ws, size_t ws_bytes, double *const *U, int trial_steps,
                         int use_graph, nmg_plan_options *best, double *times_ms, hipStream_t s)
{
    if (trial_steps < 1 || trial_steps > 100) return fail(NMG_EINVAL, "trial_steps must be in [1, 100]");
    if (!U) return fail(NMG_EINVAL, "null state array");
    if (ws_bytes < P->total) return fail(NMG_ENOMEM_WS, "workspace too small");
    // the trials move U: keep a device copy of every state
    std::vector<size_t> off(P->n + 1, 0);
    for (int k = 0; k < P->n; k++) {
        if (!U[k]) return fail(NMG_EINVAL, "null state pointer");
        off[k + 1] = off[k] + 2 * (size_t)P->insts[k].N;
    }
    double *save = nullptr;
    HIP_TRY(hipMalloc((void **)&save, sizeof(double) * off[P->n]));
    struct Free { double *p; ~Free() { if (p) (void)hipFree(p); } } guard{save};
    for (int k = 0; k < P->n; k++)
        HIP_TRY(hipMemcpyAsync(save + off[k], U[k], sizeof(double) * (off[k + 1] - off[k]),
                               hipMemcpyDeviceToDevice, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    struct FreeEv { hipEvent_t a, b; ~FreeEv() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } evg{e0, e1};
    int best_cells = P->bottom_cells, best_split = P->split_finest, best_tile = P->smooth_tile;
    int best_res = P->split_residual;
    double best_ms = 1e300;
    // candidate ci: bottom_cells = kBottomCandidates[ci % 4], split_finest = (ci / 4) % 2,
    // smooth_tile = kTileCandidates[(ci / 8) % 2], split_residual = ci / 16
    for (int ci = 0; ci < NMG_TUNE_CANDIDATES; ci++) {
        const int cells = kBottomCandidates[ci % 4], split = (ci / 4) % 2, tile = kTileCandidates[(ci / 8) % 2];
        const int sres = ci / 16;
        nmg_status st = apply_options(P, cells, split, tile, sres);
        if (st != NMG_OK) return st;
        P->n_start.assign(P->n, 0);
        if ((st = plan_begin(P, ws, ws_bytes, U, s)) != NMG_OK) return st;
        if ((st = plan_steps(P, ws, 1, use_graph, s)) != NMG_OK) return st;   // warm, capture
        HIP_TRY(hipEventRecord(e0, s));
        if ((st = plan_steps(P, ws, trial_steps, use_graph, s)) != NMG_OK) return st;
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        const double per = ms / trial_steps;
        if (times_ms) times_ms[ci] = per;
        if (per < best_ms) { best_ms = per; best_cells = cells; best_split = split; best_tile = tile; best_res = sres; }
        for (int k = 0; k < P->n; k++)
            HIP_TRY(hipMemcpyAsync(U[k], save + off[k], sizeof(double) * (off[k + 1] - off[k]),
                                   hipMemcpyDeviceToDevice, s));
    }
    nmg_status st = apply_options(P, best_cells, best_split, best_tile, best_res);
    if (st != NMG_OK) return st;
    HIP_TRY(hipStreamSynchronize(s));
    if (best) {
        memset(best, 0, sizeof(*best));
        best->bottom_cells = best_cells;
        best->fused_finest = P->fused0.second > 0 ? 1 : 0;
        best->smooth_tile = best_tile;
        best->split_finest = best_split;
        best->split_residual = best_res;
    }
    return NMG_OK;
}

}  // namespace

extern "C" {

const char *nmg_last_error(void) { return g_err.c_str(); }

nmg_status nmg_lane_stream_create(void **stream)
{
    if (!stream) return fail(NMG_EINVAL, "null argument");
    *stream = nullptr;
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (cus <= 0 || cus > 1024) return fail(NMG_EHIP, "unexpected compute-unit count");
    std::vector<uint32_t> mask((cus + 31) / 32, 0xFFFFFFFFu);
    if (cus % 32) mask.back() = (1u << (cus % 32)) - 1u;
    hipStream_t s = nullptr;
    HIP_TRY(hipExtStreamCreateWithCUMask(&s, (uint32_t)mask.size(), mask.data()));
    *stream = s;
    return NMG_OK;
}

nmg_status nmg_lane_stream_destroy(void *stream)
{
    if (!stream) return fail(NMG_EINVAL, "null stream");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    HIP_TRY(hipStreamDestroy((hipStream_t)stream));
    return NMG_OK;
}

nmg_status nmg_plan_create(const nmg_desc *descs, const nmg_params *params, int32_t n, nmg_plan **out)
{
    if (!descs || !params || !out) return fail(NMG_EINVAL, "null argument");
    if (n <= 0) return fail(NMG_EINVAL, "need at least one instance");
    nmg_plan *P = new (std::nothrow) nmg_plan();
    if (!P) return fail(NMG_EINVAL, "out of host memory");
    P->descs.assign(descs, descs + n);
    P->params.assign(params, params + n);
    // the smallest bottom threshold has the most smoothing tiles: reserve for it
    P->bottom_cells = 256;
    nmg_status st = build_plan(P, descs, params, n);
    if (st != NMG_OK) { delete P; return st; }
    P->tile_cap = P->tiles.size();
    P->bottom_cells = 2048;
    P->bottom_nt = 1024;
    st = build_plan(P, descs, params, n);
    if (st != NMG_OK) { delete P; return st; }
    *out = P;
    return NMG_OK;
}

size_t nmg_plan_workspace_bytes(const nmg_plan *plan) { return plan ? plan->total : 0; }

nmg_status nmg_plan_profile(nmg_plan *P, int32_t kernel)
{
    if (!P) return fail(NMG_EINVAL, "null plan");
    if (kernel < NMG_K_NONE || kernel > NMG_K_SMOOTH_FUSED) return fail(NMG_EINVAL, "unknown kernel id");
    P->prof_kernel = kernel;
    return NMG_OK;
}

nmg_status nmg_plan_profile_read(nmg_plan *P, double *ms, int32_t *launches)
{
    if (!P) return fail(NMG_EINVAL, "null plan");
    if (!P->ev_open.empty()) HIP_TRY(hipStreamSynchronize(P->prof_stream));
    for (auto &pr : P->ev_open) {
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, pr.first, pr.second));
        P->prof_ms += t;
        P->prof_count += 1;
        P->ev_pool.push_back(pr.first);
        P->ev_pool.push_back(pr.second);
    }
    P->ev_open.clear();
    if (ms) *ms = P->prof_ms;
    if (launches) *launches = P->prof_count;
    P->prof_ms = 0.0;
    P->prof_count = 0;
    return NMG_OK;
}

void nmg_plan_destroy(nmg_plan *plan) { delete plan; }

nmg_status nmg_plan_set_options(nmg_plan *P, const nmg_plan_options *opt)
{
    if (!P || !opt) return fail(NMG_EINVAL, "null argument");
    return apply_options(P, opt->bottom_cells, opt->split_finest, opt->smooth_tile, opt->split_residual);
}

nmg_status nmg_plan_get_options(const nmg_plan *P, nmg_plan_options *opt)
{
    if (!P || !opt) return fail(NMG_EINVAL, "null argument");
    memset(opt, 0, sizeof(*opt));
    opt->bottom_cells = P->bottom_cells;
    opt->fused_finest = P->fused0.second > 0 ? 1 : 0;
    opt->smooth_tile = P->smooth_tile;
    opt->split_finest = P->split_finest;
    opt->split_residual = P->split_residual;
    return NMG_OK;
}

nmg_status nmg_plan_autotune(nmg_plan *P, void *ws, size_t ws_bytes, double *const *U, int32_t trial_steps,
                             int32_t use_graph, nmg_plan_options *best, double *times_ms, void *stream)
{
    if (!P || !ws) return fail(NMG_EINVAL, "null plan or workspace");
    return plan_autotune(P, (char *)ws, ws_bytes, U, trial_steps, use_graph, best, times_ms,
                         (hipStream_t)stream);
}

nmg_status nmg_plan_begin(nmg_plan *P, void *ws, size_t ws_bytes, double *const *U, void *stream)
{
    if (!P) return fail(NMG_EINVAL, "null plan");
    P->n_start.assign(P->n, 0);
    return plan_begin(P, (char *)ws, ws_bytes, U, (hipStream_t)stream);
}

nmg_status nmg_plan_resume(nmg_plan *P, void *ws, size_t ws_bytes, double *const *U, const int32_t *n_done,
                           void *stream)
{
    if (!P) return fail(NMG_EINVAL, "null plan");
    if (!n_done) return fail(NMG_EINVAL, "null step counts");
    P->n_start.assign(P->n, 0);
    for (int k = 0; k < P->n; k++) {
        if (n_done[k] < 0) return fail(NMG_EINVAL, "negative step count");
        if (n_done[k] >= P->insts[k].n_max)
            return fail(NMG_EINVAL, "instance " + std::to_string(k) + " has no Newton steps left");
        P->n_start[k] = n_done[k];
    }
    return plan_begin(P, (char *)ws, ws_bytes, U, (hipStream_t)stream);
}

nmg_status nmg_plan_steps(nmg_plan *P, void *ws, int32_t steps, int32_t use_graph, int32_t *active_out,
                          nmg_stats *stats, void *stream)
{
    if (!P || !ws) return fail(NMG_EINVAL, "null plan or workspace");
    hipStream_t s = (hipStream_t)stream;
    nmg_status st = plan_steps(P, (char *)ws, steps, use_graph, s);
    if (st != NMG_OK) return st;
    if (active_out || stats) {
        st = read_state(P, (char *)ws, s ? s : P->own_stream);
        if (st != NMG_OK) return st;
        for (int k = 0; k < P->n; k++) {
            if (active_out) active_out[k] = P->host_state[k].active;
            if (stats) {
                stats[k].iters = P->host_state[k].n;
                stats[k].status = P->host_state[k].status;
                stats[k].res = P->host_state[k].res;
            }
        }
    }
    return NMG_OK;
}

nmg_status nmg_plan_solve(nmg_plan *P, void *ws, size_t ws_bytes, double *const *U, nmg_stats *stats,
                          int32_t use_graph, void *stream)
{
    if (!P) return fail(NMG_EINVAL, "null plan");
    hipStream_t s = (hipStream_t)stream;
    P->n_start.assign(P->n, 0);
    nmg_status st = plan_begin(P, (char *)ws, ws_bytes, U, s);
    if (st != NMG_OK) return st;
    int max_steps = 0;
    for (auto &I : P->insts) max_steps = std::max(max_steps, I.n_max);
    int done = 0;
    st = read_state(P, (char *)ws, s);
    if (st != NMG_OK) return st;
    for (;;) {
        bool any = false;
        for (int k = 0; k < P->n; k++) any = any || P->host_state[k].active;
        if (!any || done >= max_steps) break;
        int chunk = std::min(P->check_every, max_steps - done);
        st = plan_steps(P, (char *)ws, chunk, use_graph, s);
        if (st != NMG_OK) return st;
        done += chunk;
        st = read_state(P, (char *)ws, s ? s : (use_graph ? P->own_stream : s));
        if (st != NMG_OK) return st;
    }
    nmg_status worst = NMG_OK;
    for (int k = 0; k < P->n; k++) {
        if (stats) {
            stats[k].iters = P->host_state[k].n;
            stats[k].status = P->host_state[k].status;
            stats[k].res = P->host_state[k].res;
        }
        if (P->host_state[k].status == NMG_ENONFINITE) worst = NMG_ENONFINITE;
        else if (P->host_state[k].status == NMG_NOT_CONVERGED && worst == NMG_OK) worst = NMG_NOT_CONVERGED;
    }
    if (worst == NMG_ENONFINITE) g_err = "non-finite residual in at least one instance";
    return worst;
}

size_t nmg_workspace_bytes(const nmg_desc *desc, const nmg_params *params)
{
    if (desc && desc->dim == 2) return workspace2d_bytes(desc, params);
    nmg_plan P;
    if (build_plan(&P, desc, params, 1, false) != NMG_OK) return 0;
    return P.total;
}

nmg_status nmg_residual(const nmg_desc *desc, const double *U, double *R, double *rn,
                        double *res_dev, void *stream)
{
    if (desc && desc->dim == 2) return residual2d(desc, U, R, rn, res_dev, (hipStream_t)stream);
    nmg_params p;
    memset(&p, 0, sizeof(p));
    p.eps = 1.0; p.nu3 = 1;
    nmg_status st = check_desc1d(desc, &p);
    if (st != NMG_OK) return st;
    if (!U || !R || !rn) return fail(NMG_EINVAL, "null U/R/rn");
    Inst1D I = make_inst(desc, &p);
    I.U = const_cast<double *>(U);
    I.R = R;
    I.rn = rn;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_residual1d(nullptr, nullptr, 0, &I, nullptr, nullptr, I.recon, s));
    if (res_dev) HIP_TRY(launch_sum_res(rn, I.N, res_dev, s));
    return NMG_OK;
}

nmg_status nmg_jacobian_assemble_simplified(const nmg_desc *desc, const nmg_params *params,
                                            const double *U, const double *R, const double *rn,
                                            double *J, void *stream)
{
    if (desc && desc->dim == 2) return jacobian2d(desc, params, U, R, rn, J, (hipStream_t)stream);
    nmg_status st = check_desc1d(desc, params);
    if (st != NMG_OK) return st;
    if (!U || !R || !rn || !J) return fail(NMG_EINVAL, "null U/R/rn/J");
    Inst1D I = make_inst(desc, params);
    I.U = const_cast<double *>(U);
    I.R = const_cast<double *>(R);
    I.rn = const_cast<double *>(rn);
    MGArgs none;
    memset(&none, 0, sizeof(none));
    HIP_TRY(launch_jacobian1d(nullptr, nullptr, 0, &I, J, none, NMG_FP64, 0, I.recon, (hipStream_t)stream));
    return NMG_OK;
}

nmg_status nmg_mg_vcycle(const nmg_desc *desc, const nmg_params *params, void *ws, size_t ws_bytes,
                         const void *J, const void *rhs, void *dU, int32_t setup, void *stream)
{
    if (desc && desc->dim == 2) return vcycle2d(desc, params, ws, ws_bytes, J, rhs, dU, setup, (hipStream_t)stream);
    if (!ws || !rhs || !dU || (setup && !J)) return fail(NMG_EINVAL, "null argument");
    if (params && params->linear == NMG_LINEAR_MG_SWEEPS) return fail(NMG_EINVAL, "the directional sweeps are 2D only");
    if (params && params->linear != NMG_LINEAR_MG) return fail(NMG_EINVAL, "a V-cycle needs linear = NMG_LINEAR_MG");
    nmg_plan P;
    nmg_status st = build_plan(&P, desc, params, 1);
    if (st != NMG_OK) return st;
    if (ws_bytes < P.total) return fail(NMG_ENOMEM_WS, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    st = upload_tables(&P, w, nullptr, s);
    if (st != NMG_OK) return st;
    MGArgs mg = mg_args(&P, w, false);
    const Level1D &L0 = P.levs[0];
    const size_t vsz = P.prec == NMG_FP32_MG ? 4 : 8;
    char *mgb = w + P.off_mg;
    const long long n0 = L0.n;
    if (setup) {
        HIP_TRY(launch_convert(J, NMG_FP64, mgb + vsz * L0.J, P.prec, (long long)L0.nb * 4 * n0, s));
        st = enqueue_setup(&P, w, mg, s);
        if (st != NMG_OK) return st;
    }
    HIP_TRY(launch_convert(rhs, P.prec, mgb + vsz * L0.rhs, P.prec, 2 * n0, s));
    HIP_TRY(launch_convert(dU, P.prec, mgb + vsz * L0.dU, P.prec, 2 * n0, s));
    st = enqueue_vcycle(&P, w, mg, false, false, s);
    if (st != NMG_OK) return st;
    HIP_TRY(launch_convert(mgb + vsz * L0.dU, P.prec, dU, P.prec, 2 * n0, s));
    HIP_TRY(hipStreamSynchronize(s));   // the pinned table staging belongs to this call's plan
    return NMG_OK;
}

nmg_status nmg_interp2d_coarse_to_fine(const double *Uc, int32_t nxc, int32_t nyc, double *Uf, void *stream)
{
    if (!Uc || !Uf) return fail(NMG_EINVAL, "null argument");
    if (nxc < 3 || nyc < 3) return fail(NMG_EINVAL, "the interpolation needs at least three coarse cells in each direction");
    if ((long long)nxc * nyc > (1LL << 26) || nyc > 32767) return fail(NMG_EINVAL, "grid too large");
    HIP_TRY(launch_interp_a3(Uc, nxc, nyc, Uf, (hipStream_t)stream));
    return NMG_OK;
}

nmg_status nmg_interp_coarse_to_fine(const double *Uc, int32_t nc, double *Uf, void *stream)
{
    if (!Uc || !Uf) return fail(NMG_EINVAL, "null argument");
    if (nc < 3) return fail(NMG_EINVAL, "the interpolation needs at least three coarse cells");
    HIP_TRY(launch_interp_a2(Uc, nc, Uf, (hipStream_t)stream));
    return NMG_OK;
}

size_t nmg_nested_workspace_bytes(const nmg_desc *descs, int32_t ngrids, const nmg_params *params)
{
    if (!descs || !params || ngrids < 1 || ngrids > kMaxLevels) return 0;
    size_t m = 0;
    for (int g = 0; g < ngrids; g++) {
        const size_t b = nmg_workspace_bytes(&descs[g], &params[g]);
        if (b == 0) return 0;
        m = std::max(m, b);
    }
    return m;
}

nmg_status nmg_nested_solve(const nmg_desc *descs, int32_t ngrids, const nmg_params *params, void *ws,
                            size_t ws_bytes, double *const *U, nmg_stats *stats, void *stream)
{
    if (!descs || !params || !ws || !U || !stats) return fail(NMG_EINVAL, "null argument");
    if (ngrids < 1 || ngrids > kMaxLevels) return fail(NMG_EINVAL, "ngrids must be in [1, 16]");
    const int dim = descs[0].dim;
    if (dim != 1 && dim != 2) return fail(NMG_EINVAL, "dim must be 1 or 2");
    for (int g = 0; g < ngrids; g++) {
        if (descs[g].dim != dim) return fail(NMG_EINVAL, "every grid of a nested iteration has the same dim");
        if (!U[g]) return fail(NMG_EINVAL, "null state pointer");
        if (g > 0 && (descs[g].nx * 2 != descs[g - 1].nx || (dim == 2 && descs[g].ny * 2 != descs[g - 1].ny)))
            return fail(NMG_EINVAL, "grid g must have half the cells of grid g-1 in each direction");
        if (g > 0 && (descs[g].nx < 3 || (dim == 2 && descs[g].ny < 3)))
            return fail(NMG_EINVAL, "the interpolation needs at least three coarse cells in each direction");
        if (descs[g].levels != ngrids - g) return fail(NMG_EINVAL, "grid g must have ngrids - g levels");
    }
    if (ws_bytes < nmg_nested_workspace_bytes(descs, ngrids, params))
        return fail(NMG_ENOMEM_WS, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    for (int g = ngrids - 1; g >= 0; g--) {
        if (g < ngrids - 1) {
            if (dim == 1) HIP_TRY(launch_interp_a2(U[g + 1], descs[g + 1].nx, U[g], s));
            else HIP_TRY(launch_interp_a3(U[g + 1], descs[g + 1].nx, descs[g + 1].ny, U[g], s));
        }
        const nmg_status st = nmg_newton_solve(&descs[g], &params[g], ws, ws_bytes, U[g], &stats[g],
                                               nullptr, 0, stream);
        if (st < 0 && st != NMG_ENONFINITE) return st;
        if (stats[g].status == NMG_ENONFINITE) return fail(NMG_ENONFINITE, "grid " + std::to_string(g) + " diverged");
    }
    return stats[0].status;
}

nmg_status nmg_autotune2d(const nmg_desc *desc, const nmg_params *params, void *ws, size_t ws_bytes,
                          const double *J, const void *rhs, int32_t cycles, int32_t *best, double *ms, void *stream)
{
    if (!desc || desc->dim != 2 || !params) return fail(NMG_EINVAL, "nmg_autotune2d takes a 2D problem");
    return autotune2d(desc, params, ws, ws_bytes, J, rhs, cycles, best, ms, (hipStream_t)stream);
}

nmg_status nmg_newton2d_begin(const nmg_desc *desc, const nmg_params *params, void *ws, size_t ws_bytes,
                              double *U, void *stream)
{
    if (!desc || desc->dim != 2) return fail(NMG_EINVAL, "nmg_newton2d_begin takes a 2D problem");
    return newton2d_begin(desc, params, ws, ws_bytes, U, (hipStream_t)stream);
}

nmg_status nmg_newton2d_steps(const nmg_desc *desc, const nmg_params *params, void *ws, size_t ws_bytes,
                              double *U, int32_t steps, nmg_newton_state *state_out, void *stream)
{
    if (!desc || desc->dim != 2) return fail(NMG_EINVAL, "nmg_newton2d_steps takes a 2D problem");
    return newton2d_steps(desc, params, ws, ws_bytes, U, steps, state_out, (hipStream_t)stream);
}

nmg_status nmg_newton_solve(const nmg_desc *desc, const nmg_params *params, void *ws, size_t ws_bytes,
                            double *U, nmg_stats *stats, double *hist, int32_t max_hist, void *stream)
{
    if (desc && desc->dim == 2) {
        nmg_stats local;
        return newton2d(desc, params, ws, ws_bytes, U, stats ? stats : &local, hist, max_hist, (hipStream_t)stream);
    }
    nmg_plan P;
    nmg_status st = build_plan(&P, desc, params, 1);
    if (st != NMG_OK) return st;
    double *Us[1] = {U};
    nmg_stats local;
    st = nmg_plan_solve(&P, ws, ws_bytes, Us, stats ? stats : &local, params->check_every > 1 ? 1 : 0,
                        stream);
    if (hist && max_hist > 0) {
        nmg_stats &S = stats ? *stats : local;
        int cnt = std::min(std::min((int)max_hist, S.iters), P.max_hist);
        if (cnt > 0) {
            hipStream_t s = (hipStream_t)stream;
            if (hipMemcpyAsync(hist, (char *)ws + P.off_hist, sizeof(double) * cnt, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return fail(NMG_EHIP, "history copy failed");
        }
    }
    return st;
}

}  // extern "C"

// ---- the Newton solve that allocates nothing -----------------------------------------------

namespace {

constexpr size_t kStaticWsBytes = size_t(NMG_STATIC_WS_MIB) << 20;
constexpr int kMaxDevices = 64;

}  // namespace

// The library's own device workspace for nmg_newton_solve_static.  Every GPU the library runs on
// holds its own copy from the library's load until the process ends.  In host code the name is
// only a stand-in for the symbol: the array's device address comes from hipGetSymbolAddress.
static __device__ __align__(256) char scratch[kStaticWsBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// this device's address of `scratch`, looked up once per device (with that device current)
nmg_status scratch_address(void **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(NMG_EHIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(NMG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return NMG_OK;
}

}  // namespace

extern "C" {

nmg_status nmg_newton_solve_static(const nmg_desc *desc, const nmg_params *params, double *U,
                                   nmg_stats *stats, double *hist, int32_t max_hist, void *stream)
{
    if (!desc || !params) return fail(NMG_EINVAL, "null desc or params");
    if (!U) return fail(NMG_EINVAL, "null U");
    const size_t need = nmg_workspace_bytes(desc, params);
    if (need == 0) return NMG_EINVAL;   // the size query has set the message
    if (need > kStaticWsBytes)
        return fail(NMG_ENOMEM_WS, "the problem needs " + std::to_string(need) +
                                       " bytes of workspace; the static workspace holds " +
                                       std::to_string(kStaticWsBytes) + " (use nmg_newton_solve)");
    void *ws = nullptr;
    nmg_status st = scratch_address(&ws);
    if (st != NMG_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    nmg_stats local;
    nmg_stats &S = stats ? *stats : local;
    if (desc->dim == 2) return newton2d(desc, params, ws, kStaticWsBytes, U, &S, hist, max_hist, s);
    nmg_plan P;
    st = build_plan(&P, desc, params, 1);
    if (st != NMG_OK) return st;
    // the instance table and the Newton state pass through host buffers on this call's stack
    // instead of pinned allocations; the call synchronises before they go out of scope
    alignas(64) char tables[sizeof(Inst1D)];
    NewtonState hs;
    P.host_tables = tables;
    P.host_state = &hs;
    P.host_borrowed = true;
    double *Us[1] = {U};
    st = nmg_plan_solve(&P, ws, kStaticWsBytes, Us, &S, 0, stream);
    if (hist && max_hist > 0 && (st >= 0 || st == NMG_ENONFINITE)) {
        const int cnt = std::min(std::min((int)max_hist, S.iters), P.max_hist);
        if (cnt > 0) {
            if (hipMemcpyAsync(hist, (char *)ws + P.off_hist, sizeof(double) * cnt, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                return fail(NMG_EHIP, "history copy failed");
        }
    }
    return st;
}

}  // extern "C"
