// Batched stepping of several independent scenes (the serving form of the
// step; see include/flip.h). Host side only: the kernels are the plain
// step's kernels in their batched form (batch.h). Every launch of the step
// covers all scenes; each scene keeps its own workspace, reductions and
// convergence test, so a scene's result does not depend on its batch.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/flip.h"
#include "batch.h"
#include "common.h"
#include "handle.h"

using namespace flipmi;

namespace {

constexpr size_t TABLE_ALIGN = 256;
constexpr int GRAPH_CHUNK = 8;  // solver iterations per recorded chunk (even: direction buffers alternate)
constexpr int FIRST_CHUNK = 16; // solver iterations before the first convergence check, without history
constexpr int NEXT_CHUNK = 8;   // solver iterations between later checks
// Multigrid batches: an iteration launched past convergence costs fourteen
// launches, so they start with the previous step's largest count and then
// test every MG_NEXT_CHUNK iterations (a recorded chunk of that size too).
constexpr int MG_NEXT_CHUNK = 2;

// Host image of the launch tables, uploaded once into the batch workspace.
struct Tables {
    std::vector<char> bytes;
    // reserve n zeroed bytes, aligned
    size_t reserve(size_t n)
    {
        const size_t o = (bytes.size() + TABLE_ALIGN - 1) & ~(TABLE_ALIGN - 1);
        bytes.resize(o + (n ? n : 1), 0);
        return o;
    }
    size_t put(const void* p, size_t n)
    {
        const size_t o = reserve(n);
        std::memcpy(bytes.data() + o, p, n);
        return o;
    }
};

// one batched launch: offsets of its tables in the workspace
struct Site {
    size_t args_off = 0, first_off = 0;
    int ns = 0;
    uint32_t blocks = 0;
    uint64_t items = 0;  // work-items of the launch
};

template <typename A>
Site add_site(Tables& t, const std::vector<A>& args, const std::vector<uint32_t>& blocks, int threads)
{
    std::vector<uint32_t> first(args.size() + 1, 0u);
    uint64_t total = 0;
    for (size_t i = 0; i < args.size(); ++i) {
        total += blocks[i];
        first[i + 1] = (uint32_t)std::min<uint64_t>(total, 0xFFFFFFFFull);
    }
    Site s;
    s.args_off = t.put(args.data(), sizeof(A) * args.size());
    s.first_off = t.put(first.data(), sizeof(uint32_t) * first.size());
    s.ns = (int)args.size();
    s.blocks = first.back();
    s.items = total * (uint64_t)threads;
    return s;
}

// launches whose arguments depend on which particle buffer is current
struct PhaseSites {
    Site bin_keys, gather, p2g, g2p;
};

struct Sites {
    Site fill_count, scan_c[3], scatter, tile_flags, scan_t[3], tile_compact, rhs, dir[2], upd[2], project[3],
        summary;
    PhaseSites ph[2];
    size_t summary_off = 0;  // SolveSummary[ns]
    // multigrid (all scenes or none): levels below the fine grid, deepest scene
    bool mg = false;
    int mg_levels = 0;
    Site mg_types_fine, mg_fine_down, mg_fine_up, mg_bottom;
    Site mg_types[MG_MAX_LEVELS], mg_down[MG_MAX_LEVELS], mg_up[MG_MAX_LEVELS];
};

template <typename T>
void scan_sites(Tables& t, const std::vector<const uint32_t*>& in, const std::vector<uint32_t*>& out,
                const std::vector<int64_t>& n, const std::vector<uint32_t*>& tmp, Site site[3])
{
    const size_t ns = in.size();
    std::vector<ScanTotalsArgs> a0(ns);
    std::vector<ScanTotalsScanArgs> a1(ns);
    std::vector<ScanApplyArgs> a2(ns);
    std::vector<uint32_t> b0(ns), b1(ns);
    for (size_t s = 0; s < ns; ++s) {
        const int64_t nb = n[s] > 0 ? scan_blocks(n[s]) : 0;
        a0[s] = ScanTotalsArgs{in[s], n[s], tmp[s]};
        a1[s] = ScanTotalsScanArgs{tmp[s], nb};
        a2[s] = ScanApplyArgs{in[s], out[s], n[s], tmp[s]};
        b0[s] = (uint32_t)nb;
        b1[s] = nb > 0 ? 1u : 0u;
    }
    site[0] = add_site(t, a0, b0, SCAN_NT);
    site[1] = add_site(t, a1, b1, 1024);
    site[2] = add_site(t, a2, b0, SCAN_NT);
}

// The tables of every launch of one step, with the same arguments and grids
// as the plain step of each handle (capi.hip, run_step).
template <typename T>
void build_sites(const std::vector<flip_handle*>& hs, Tables& t, Sites& S)
{
    const size_t ns = hs.size();
    std::vector<uint32_t> blk(ns);
    {
        std::vector<FillU32Args> a(ns);
        for (size_t s = 0; s < ns; ++s) {
            a[s] = FillU32Args{hs[s]->count, hs[s]->sz.C, 0u};
            blk[s] = elem_blocks(hs[s]->sz.C);
        }
        S.fill_count = add_site(t, a, blk, ELEM_NT);
    }
    for (int ph = 0; ph < 2; ++ph) {
        std::vector<BinKeysArgs<T>> ak(ns);
        std::vector<GatherArgs<T>> ag(ns);
        std::vector<P2GArgs<T>> ap(ns);
        std::vector<G2PArgs<T>> a2(ns);
        std::vector<uint32_t> bp(ns), bt(ns), b2g(ns);
        for (size_t s = 0; s < ns; ++s) {
            flip_handle* h = hs[s];
            const Geo& g = h->geo;
            const flip_config& c = h->cfg;
            const int64_t n = h->sz.n;
            const int cur = h->cur ^ ph, nxt = cur ^ 1;
            const T* pc = (const T*)h->pos[cur];
            ak[s] = BinKeysArgs<T>{g, pc, pc + n, pc + 2 * n, n, h->key, h->rank, h->count};
            ag[s] = GatherArgs<T>{h->perm, h->key, h->start, h->count, n,
                                  (const T*)h->pos[cur], (const T*)h->vel[cur], h->id[cur],
                                  (T*)h->pos[nxt], (T*)h->vel[nxt], h->id[nxt]};
            T* pn = (T*)h->pos[nxt];
            T* vn = (T*)h->vel[nxt];
            const bool grav = !(c.flags & FLIP_FLAG_NO_GRAVITY);
            P2GArgs<T> p;
            p.g = g;
            p.n = n;
            p.px = pn;
            p.py = pn + n;
            p.pz = pn + 2 * n;
            p.vx = vn;
            p.vy = vn + n;
            p.vz = vn + 2 * n;
            p.start = h->start;
            p.count = h->count;
            p.tile_flag = h->tile_flag;
            for (int a = 0; a < 3; ++a) {
                p.gdt[a] = (T)(grav ? c.gravity[a] * c.dt : 0.0);
                p.old[a] = (T*)h->f_old[a];
                p.star[a] = (T*)h->f_star[a];
            }
            ap[s] = p;
            G2PArgs<T> q;
            q.g = g;
            q.n = n;
            q.start = h->start;
            q.count = h->count;
            q.px = pn;
            q.py = pn + n;
            q.pz = pn + 2 * n;
            q.vx = vn;
            q.vy = vn + n;
            q.vz = vn + 2 * n;
            q.un = (const T*)h->f_new[0];
            q.vn = (const T*)h->f_new[1];
            q.wn = (const T*)h->f_new[2];
            q.uo = (const T*)h->f_old[0];
            q.vo = (const T*)h->f_old[1];
            q.wo = (const T*)h->f_old[2];
            q.alpha = (T)c.flip_ratio;
            q.dt = (T)c.dt;
            q.skin = (T)(1e-3 * g.dx);
            q.Lx = (T)(g.nx * g.dx);
            q.Ly = (T)(g.ny * g.dx);
            q.Lz = (T)(g.nz * g.dx);
            q.advect_particle_vel = (c.flags & FLIP_FLAG_ADVECT_PARTICLE_VEL) ? 1 : 0;
            q.nonfinite = &h->diagw->nonfinite;
            a2[s] = q;
            bp[s] = elem_blocks(n);
            bt[s] = (uint32_t)h->sz.T;
            b2g[s] = (uint32_t)p2g_blocks(g);
        }
        S.ph[ph].bin_keys = add_site(t, ak, bp, ELEM_NT);
        S.ph[ph].gather = add_site(t, ag, bp, ELEM_NT);
        S.ph[ph].p2g = add_site(t, ap, b2g, P2G_NT);
        S.ph[ph].g2p = add_site(t, a2, bt, 256);
    }
    {
        std::vector<const uint32_t*> in(ns);
        std::vector<uint32_t*> out(ns), tmp(ns);
        std::vector<int64_t> n(ns);
        for (size_t s = 0; s < ns; ++s) {
            in[s] = hs[s]->count;
            out[s] = hs[s]->start;
            n[s] = hs[s]->sz.C;
            tmp[s] = hs[s]->scan_tmp;
        }
        scan_sites<T>(t, in, out, n, tmp, S.scan_c);
        for (size_t s = 0; s < ns; ++s) {
            in[s] = hs[s]->tile_flag;
            out[s] = hs[s]->tile_excl;
            n[s] = hs[s]->sz.T;
        }
        scan_sites<T>(t, in, out, n, tmp, S.scan_t);
    }
    {
        std::vector<ScatterArgs> a(ns);
        std::vector<TileFlagsArgs> f(ns);
        std::vector<TileCompactArgs> k(ns);
        std::vector<uint32_t> bp(ns), bt(ns), bc(ns);
        for (size_t s = 0; s < ns; ++s) {
            flip_handle* h = hs[s];
            a[s] = ScatterArgs{h->key, h->rank, h->start, h->sz.n, h->perm};
            f[s] = TileFlagsArgs{h->geo, h->count, h->tile_flag};
            k[s] = TileCompactArgs{h->geo, h->tile_flag, h->tile_excl, h->tile_slot, h->tile_list, h->tile_nbr,
                                   h->d_nactive};
            bp[s] = elem_blocks(h->sz.n);
            bt[s] = (uint32_t)h->sz.T;
            bc[s] = elem_blocks(h->sz.T);
        }
        S.scatter = add_site(t, a, bp, ELEM_NT);
        S.tile_flags = add_site(t, f, bt, 256);
        S.tile_compact = add_site(t, k, bc, ELEM_NT);
    }
    {
        std::vector<RhsArgs<T, T>> r(ns);
        std::vector<DirArgs<T>> d0(ns), d1(ns);
        std::vector<UpdArgs<T>> u0(ns), u1(ns);
        std::vector<ProjectArgs<T, T>> pr[3];
        for (auto& v : pr) v.resize(ns);
        std::vector<uint32_t> bg(ns), bf[3];
        for (auto& v : bf) v.resize(ns);
        for (size_t s = 0; s < ns; ++s) {
            flip_handle* h = hs[s];
            const flip_config& c = h->cfg;
            RhsArgs<T, T> q;
            q.g = h->geo;
            q.tile_list = h->tile_list;
            q.d_nactive = h->d_nactive;
            q.count = h->count;
            q.u = (const T*)h->f_star[0];
            q.v = (const T*)h->f_star[1];
            q.w = (const T*)h->f_star[2];
            q.scale = -c.density * c.dx / c.dt;
            q.diag = h->diag;
            q.b = (T*)h->b;
            q.z = (T*)h->z;
            q.x = (T*)h->xin[0];
            q.s0 = (T*)h->s[0];
            q.s1 = (T*)h->s[1];
            q.partials = h->partials;
            q.pstride = h->groups;
            q.ps = h->ps;
            q.tol = c.pcg_tol;
            q.max_iters = solve_iter_cap(c);
            q.r_form = S.mg ? 1 : 0;
            r[s] = q;
            // with multigrid the direction kernel reads z = M r (h->z holds r)
            const T* zdir = (const T*)(S.mg ? h->mgz : h->z);
            for (int k = 0; k < 2; ++k) {
                DirArgs<T> d{-1, h->tile_nbr, h->diag, zdir, (const T*)h->s[k], (T*)h->s[k ^ 1], h->pslots,
                             h->ps};
                UpdArgs<T> u{-1, h->tile_nbr, h->diag, (const T*)h->s[k ^ 1], (T*)h->xin[0], (T*)h->z, h->pslots,
                             h->ps};
                (k ? d1 : d0)[s] = d;
                (k ? u1 : u0)[s] = u;
            }
            const T scale = (T)(c.dt / (c.density * c.dx));
            for (int a = 0; a < 3; ++a) {
                pr[a][s] = ProjectArgs<T, T>{h->geo, h->diag, h->tile_slot, (const T*)h->xin[0],
                                             (const T*)h->f_star[a], (T*)h->f_new[a], scale};
                bf[a][s] = elem_blocks(h->sz.F[a]);
            }
            bg[s] = (uint32_t)h->groups;
        }
        S.rhs = add_site(t, r, bg, TILE_CELLS);
        S.dir[0] = add_site(t, d0, bg, 256);
        S.dir[1] = add_site(t, d1, bg, 256);
        S.upd[0] = add_site(t, u0, bg, 256);
        S.upd[1] = add_site(t, u1, bg, 256);
        for (int a = 0; a < 3; ++a) S.project[a] = add_site(t, pr[a], bf[a], ELEM_NT);
    }
    if (S.mg) {
        // batched launches run every block of a level (no block lists)
        auto unlisted = [](MgLevel lv) {
            lv.uflag = lv.dlist = lv.ulist = lv.cnt = nullptr;
            return lv;
        };
        int L = 0;
        for (flip_handle* h : hs) L = std::max(L, h->nmg);
        S.mg_levels = L;
        std::vector<MgTypesFineArgs> tf(ns);
        std::vector<MgFineArgs<T>> fd(ns), fu(ns);
        std::vector<MgPairArgs> bo(ns);
        std::vector<uint32_t> btf(ns), bfine(ns), bbot(ns, 1u);
        for (size_t s = 0; s < ns; ++s) {
            flip_handle* h = hs[s];
            const MgLevel l0 = unlisted(h->mg[0]);
            tf[s] = MgTypesFineArgs{h->geo, h->tile_slot, h->diag, l0};
            btf[s] = (uint32_t)mg_blocks(MG_B_TYPES, l0, l0);
            fd[s] = MgFineArgs<T>{-1, h->geo, h->tile_list, h->tile_nbr, h->diag, (const T*)h->z, l0, nullptr,
                                  nullptr, h->ps};
            fu[s] = MgFineArgs<T>{-1, h->geo, h->tile_list, h->tile_nbr, h->diag, (const T*)h->z, l0, (T*)h->mgz,
                                  h->pslots, h->ps};
            bfine[s] = (uint32_t)h->groups;
            bo[s] = MgPairArgs{unlisted(h->mg[h->nmg - 1]), unlisted(h->mg[h->nmg - 1]), h->ps};
        }
        S.mg_types_fine = add_site(t, tf, btf, 256);
        S.mg_fine_down = add_site(t, fd, bfine, 256);
        S.mg_fine_up = add_site(t, fu, bfine, 256);
        S.mg_bottom = add_site(t, bo, bbot, 512);
        for (int l = 0; l + 1 < L; ++l) {
            // level l to l + 1, for the scenes that have both
            std::vector<MgPairArgs> a(ns);
            std::vector<uint32_t> bt(ns, 0u), bd(ns, 0u), bu(ns, 0u);
            for (size_t s = 0; s < ns; ++s) {
                flip_handle* h = hs[s];
                const bool has = l + 1 < h->nmg;
                const MgLevel f = unlisted(h->mg[has ? l : 0]);
                const MgLevel c = unlisted(h->mg[has ? l + 1 : 0]);
                a[s] = MgPairArgs{f, c, h->ps};
                if (!has) continue;
                bt[s] = (uint32_t)mg_blocks(MG_B_TYPES, f, c);
                bd[s] = (uint32_t)mg_blocks(MG_B_DOWN, f, c);
                bu[s] = (uint32_t)mg_blocks(MG_B_UP, f, c);
            }
            S.mg_types[l] = add_site(t, a, bt, 256);
            S.mg_down[l] = add_site(t, a, bd, MG_BATCH_NT);
            S.mg_up[l] = add_site(t, a, bu, MG_BATCH_NT);
        }
    }
    {
        // the summary array itself, then the summary launch that fills it
        S.summary_off = t.reserve(sizeof(SolveSummary) * ns);
        std::vector<SummaryArgs> a(ns);
        std::vector<uint32_t> b1(ns, 1u);
        for (size_t s = 0; s < ns; ++s) a[s] = SummaryArgs{hs[s]->ps, nullptr};  // rebased at create
        S.summary = add_site(t, a, b1, 64);
    }
}

bool sites_fit(const Sites& S)
{
    auto ok = [](const Site& s) { return s.items < 0xFFFFFFFFull; };
    bool r = ok(S.fill_count) && ok(S.scatter) && ok(S.tile_flags) && ok(S.tile_compact) && ok(S.rhs) &&
             ok(S.summary);
    for (int i = 0; i < 3; ++i) r = r && ok(S.scan_c[i]) && ok(S.scan_t[i]) && ok(S.project[i]);
    for (int k = 0; k < 2; ++k)
        r = r && ok(S.dir[k]) && ok(S.upd[k]) && ok(S.ph[k].bin_keys) && ok(S.ph[k].gather) && ok(S.ph[k].p2g) &&
            ok(S.ph[k].g2p);
    if (S.mg) {
        r = r && ok(S.mg_types_fine) && ok(S.mg_fine_down) && ok(S.mg_fine_up) && ok(S.mg_bottom);
        for (int l = 0; l + 1 < S.mg_levels; ++l) r = r && ok(S.mg_types[l]) && ok(S.mg_down[l]) && ok(S.mg_up[l]);
    }
    return r;
}

flip_status check_handles(flip_handle* const* handles, int nscenes, int* prec, bool* mg)
{
    if (!handles || nscenes < 1 || nscenes > FLIP_BATCH_MAX_SCENES) return FLIP_E_INVALID;
    for (int s = 0; s < nscenes; ++s) {
        const flip_handle* h = handles[s];
        if (!h) return FLIP_E_INVALID;
        if (h->prec != FLIP_FP32 && h->prec != FLIP_FP64) return FLIP_E_INVALID;
        if (h->prec != handles[0]->prec) return FLIP_E_INVALID;
        if (h->cfg.flags &
            (FLIP_FLAG_NO_PROJECTION | FLIP_FLAG_KERNEL_TIMING | FLIP_FLAG_DIAGNOSTICS | FLIP_FLAG_RED_BLACK_GS | FLIP_FLAG_ADAPTIVE_DT |
             FLIP_FLAG_RESEED))
            return FLIP_E_INVALID;
        // the preconditioner is the same for every scene of a batch
        if ((h->cfg.flags & FLIP_FLAG_MULTIGRID) != (handles[0]->cfg.flags & FLIP_FLAG_MULTIGRID))
            return FLIP_E_INVALID;
        for (int q = 0; q < s; ++q)
            if (handles[q] == h) return FLIP_E_INVALID;
    }
    *prec = handles[0]->prec;
    *mg = (handles[0]->cfg.flags & FLIP_FLAG_MULTIGRID) != 0;
    return FLIP_OK;
}

flip_status build_tables(const std::vector<flip_handle*>& hs, int prec, bool mg, Tables& t, Sites& S)
{
    S.mg = mg;
    if (prec == FLIP_FP64)
        build_sites<double>(hs, t, S);
    else
        build_sites<float>(hs, t, S);
    return sites_fit(S) ? FLIP_OK : FLIP_E_INVALID;
}

}  // namespace

struct flip_batch {
    std::vector<flip_handle*> hs;
    std::vector<int> cur0;  // each scene's current particle buffer at creation
    int prec = FLIP_FP32;
    uint32_t flags = 0;
    char* dws = nullptr;
    Sites S;
    SolveSummary* h_sum = nullptr;  // pinned host copy of the summaries
    int phase = 0;                  // steps taken, mod 2
    int64_t steps = 0;
    int max_cap = 0;                // largest iteration cap of the scenes
    hipStream_t cap_stream = nullptr;
    hipStream_t last_stream = nullptr;  // stream of the last step
    hipGraphExec_t g_pre[2] = {nullptr, nullptr};
    hipGraphExec_t g_chunk = nullptr;
    hipGraphExec_t g_chunk_small = nullptr;  // MG_NEXT_CHUNK iterations (multigrid batches)
    hipGraphExec_t g_post[2] = {nullptr, nullptr};
};

namespace {

BatchLaunch L(const flip_batch* b, const Site& s)
{
    BatchLaunch l;
    l.args = b->dws + s.args_off;
    l.first = (const uint32_t*)(b->dws + s.first_off);
    l.ns = s.ns;
    l.blocks = s.blocks;
    return l;
}

// one multigrid V-cycle z = M r of every scene: the restrictions level by
// level down to the deepest scene's coarsest level, every scene's coarsest
// sweeps, then the prolongations back up (a scene takes part in the level
// launches it has, so its own order is down, bottom, up)
template <typename T>
void enqueue_vcycle(const flip_batch* b, hipStream_t st)
{
    const Sites& S = b->S;
    launch_b_mg_fine<T>(false, L(b, S.mg_fine_down), st);
    for (int l = 0; l + 1 < S.mg_levels; ++l) launch_b_mg_level<T>(MG_B_DOWN, L(b, S.mg_down[l]), st);
    launch_b_mg_level<T>(MG_B_BOTTOM, L(b, S.mg_bottom), st);
    for (int l = S.mg_levels - 2; l >= 0; --l) launch_b_mg_level<T>(MG_B_UP, L(b, S.mg_up[l]), st);
    launch_b_mg_fine<T>(true, L(b, S.mg_fine_up), st);
}

// binning, tiles, particle-to-grid and the solver start of every scene
template <typename T>
void enqueue_pre(const flip_batch* b, int ph, hipStream_t st)
{
    const Sites& S = b->S;
    launch_b_fill_u32(L(b, S.fill_count), st);
    launch_b_bin_keys<T>(L(b, S.ph[ph].bin_keys), st);
    launch_b_scan_totals(L(b, S.scan_c[0]), st);
    launch_b_scan_totals_scan(L(b, S.scan_c[1]), st);
    launch_b_scan_apply(L(b, S.scan_c[2]), st);
    launch_b_bin_scatter(L(b, S.scatter), st);
    launch_b_bin_gather<T>(L(b, S.ph[ph].gather), st);
    launch_b_tile_flags(L(b, S.tile_flags), st);
    launch_b_scan_totals(L(b, S.scan_t[0]), st);
    launch_b_scan_totals_scan(L(b, S.scan_t[1]), st);
    launch_b_scan_apply(L(b, S.scan_t[2]), st);
    launch_b_tile_compact(L(b, S.tile_compact), st);
    launch_b_p2g<T>(L(b, S.ph[ph].p2g), st);
    launch_b_rhs<T, T>(L(b, S.rhs), st);
    if (S.mg) {
        launch_b_mg_types_fine(L(b, S.mg_types_fine), st);
        for (int l = 0; l + 1 < S.mg_levels; ++l) launch_b_mg_types(L(b, S.mg_types[l]), st);
        enqueue_vcycle<T>(b, st);
    }
    launch_b_pcg_direction<T>(L(b, S.dir[0]), st);  // D_0
}

// `iters` solver iterations from an even iteration index k: the pairs
// (U_k, D_{k+1}) (each direction kernel tests the residual the update before
// it left), then the summaries
template <typename T>
void enqueue_chunk(const flip_batch* b, int iters, hipStream_t st)
{
    const Sites& S = b->S;
    for (int i = 0; i < iters; ++i) {
        launch_b_pcg_update<T>(S.mg, L(b, S.upd[i & 1]), st);
        if (S.mg) enqueue_vcycle<T>(b, st);
        launch_b_pcg_direction<T>(L(b, S.dir[(i + 1) & 1]), st);
    }
    launch_b_summary(L(b, S.summary), st);
}

template <typename T>
void enqueue_post(const flip_batch* b, int ph, hipStream_t st)
{
    const Sites& S = b->S;
    for (int a = 0; a < 3; ++a) launch_b_project<T, T>(a, L(b, S.project[a]), st);
    launch_b_g2p<T>(L(b, S.ph[ph].g2p), st);
}

template <typename F>
flip_status record_graph(flip_batch* b, F&& enqueue, hipGraphExec_t* out)
{
    if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed));
    enqueue(b->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (e != hipSuccess || !g) return FLIP_E_HIP;
    const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return FLIP_E_HIP;
    return hipGetLastError() == hipSuccess ? FLIP_OK : FLIP_E_HIP;
}

template <typename T>
flip_status batch_step(flip_batch* b, hipStream_t st)
{
    const int ns = (int)b->hs.size();
    const int ph = b->phase;
    b->last_stream = st;
    for (int s = 0; s < ns; ++s)
        if (b->hs[s]->cur != (b->cur0[s] ^ ph)) return FLIP_E_STATE;  // stepped outside the batch
    const bool graphs = (b->flags & FLIP_BATCH_GRAPHS) && b->steps >= 1;
    if (graphs) {
        if (!b->g_pre[ph]) {
            flip_status r = record_graph(b, [&](hipStream_t cs) { enqueue_pre<T>(b, ph, cs); }, &b->g_pre[ph]);
            if (r != FLIP_OK) return r;
        }
        if (!b->g_chunk) {
            flip_status r = record_graph(b, [&](hipStream_t cs) { enqueue_chunk<T>(b, GRAPH_CHUNK, cs); },
                                         &b->g_chunk);
            if (r != FLIP_OK) return r;
        }
        if (b->S.mg && !b->g_chunk_small) {
            flip_status r = record_graph(b, [&](hipStream_t cs) { enqueue_chunk<T>(b, MG_NEXT_CHUNK, cs); },
                                         &b->g_chunk_small);
            if (r != FLIP_OK) return r;
        }
        if (!b->g_post[ph]) {
            flip_status r = record_graph(b, [&](hipStream_t cs) { enqueue_post<T>(b, ph, cs); }, &b->g_post[ph]);
            if (r != FLIP_OK) return r;
        }
        HIP_TRY(hipGraphLaunch(b->g_pre[ph], st));
    } else {
        enqueue_pre<T>(b, ph, st);
    }

    // the solve: chunks of iterations until no scene is running
    int prev = 0;
    for (flip_handle* h : b->hs) prev = std::max(prev, h->prev_iters);
    const bool mg = b->S.mg;
    int chunk = prev > 2 ? (mg ? prev : prev - 2) : FIRST_CHUNK;
    const int unit = graphs && !mg ? GRAPH_CHUNK : 2;
    chunk = (chunk + unit - 1) / unit * unit;
    int launched = 0;
    const size_t sum_bytes = sizeof(SolveSummary) * ns;
    for (;;) {
        if (graphs) {
            for (int q = 0; q < chunk / GRAPH_CHUNK; ++q) HIP_TRY(hipGraphLaunch(b->g_chunk, st));
            for (int q = 0; q < (chunk % GRAPH_CHUNK) / MG_NEXT_CHUNK; ++q)
                HIP_TRY(hipGraphLaunch(b->g_chunk_small, st));
        } else {
            enqueue_chunk<T>(b, chunk, st);
        }
        launched += chunk;
        HIP_TRY(hipMemcpyAsync(b->h_sum, b->dws + b->S.summary_off, sum_bytes, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        bool running = false;
        for (int s = 0; s < ns; ++s) running = running || b->h_sum[s].done == PCG_RUNNING;
        if (!running || launched > b->max_cap + 8) break;
        chunk = mg ? MG_NEXT_CHUNK : (graphs ? GRAPH_CHUNK : NEXT_CHUNK);
    }

    if (graphs)
        HIP_TRY(hipGraphLaunch(b->g_post[ph], st));
    else
        enqueue_post<T>(b, ph, st);
    if (hipGetLastError() != hipSuccess) return FLIP_E_HIP;

    flip_status first = FLIP_OK;
    for (int s = 0; s < ns; ++s) {
        flip_handle* h = b->hs[s];
        const SolveSummary& q = b->h_sum[s];
        flip_status ret = FLIP_OK;
        if (q.done == PCG_MAX_ITERS || q.done == PCG_RUNNING) ret = FLIP_E_NOT_CONVERGED;
        if (q.done == PCG_BREAKDOWN) ret = q.sync_error ? FLIP_E_HIP : FLIP_E_NONFINITE;
        const int status = q.done == PCG_CONVERGED ? 0 : (q.done == PCG_BREAKDOWN ? 2 : 1);
        record_step(h, q.n_active > 0, status, q.n_active, q.nfluid, q.max_b, q.max_r, q.iter, 0, ret);
        h->prev_iters = q.iter;
        h->cur ^= 1;
        h->scur = (q.iter & 1);
        h->xi = 0;
        h->last_stream = st;
        if (ret != FLIP_OK && first == FLIP_OK) first = ret;
    }
    b->phase ^= 1;
    b->steps += 1;
    return first;
}

}  // namespace

extern "C" {

flip_status flip_batch_workspace_bytes(flip_handle* const* handles, int nscenes, size_t* out_bytes)
{
    if (!out_bytes) return FLIP_E_INVALID;
    int prec = FLIP_FP32;
    bool mg = false;
    flip_status v = check_handles(handles, nscenes, &prec, &mg);
    if (v != FLIP_OK) return v;
    std::vector<flip_handle*> hs(handles, handles + nscenes);
    Tables t;
    Sites S;
    v = build_tables(hs, prec, mg, t, S);
    if (v != FLIP_OK) return v;
    *out_bytes = t.bytes.size();
    return FLIP_OK;
}

flip_status flip_batch_create(flip_handle* const* handles, int nscenes, uint32_t flags, void* d_ws,
                              size_t ws_bytes, void* hip_stream, flip_batch** out)
{
    if (!out) return FLIP_E_INVALID;
    *out = nullptr;
    if (flags & ~(uint32_t)FLIP_BATCH_GRAPHS) return FLIP_E_INVALID;
    int prec = FLIP_FP32;
    bool mg = false;
    flip_status v = check_handles(handles, nscenes, &prec, &mg);
    if (v != FLIP_OK) return v;
    flip_batch* b = new (std::nothrow) flip_batch();
    if (!b) return FLIP_E_INVALID;
    b->hs.assign(handles, handles + nscenes);
    b->prec = prec;
    b->flags = flags;
    Tables t;
    v = build_tables(b->hs, prec, mg, t, b->S);
    if (v != FLIP_OK) {
        delete b;
        return v;
    }
    if (!d_ws || ws_bytes < t.bytes.size() || ((uintptr_t)d_ws & (TABLE_ALIGN - 1))) {
        delete b;
        return FLIP_E_WORKSPACE;
    }
    b->dws = (char*)d_ws;
    // the summary launch writes scene s's entry of the summary array
    SummaryArgs* sa = (SummaryArgs*)(t.bytes.data() + b->S.summary.args_off);
    SolveSummary* d_sum = (SolveSummary*)(b->dws + b->S.summary_off);
    for (int s = 0; s < nscenes; ++s) sa[s].out = d_sum + s;
    for (flip_handle* h : b->hs) {
        b->cur0.push_back(h->cur);
        b->max_cap = std::max(b->max_cap, solve_iter_cap(h->cfg));
    }
    hipStream_t st = (hipStream_t)hip_stream;
    if (hipHostMalloc((void**)&b->h_sum, sizeof(SolveSummary) * nscenes, hipHostMallocDefault) != hipSuccess ||
        hipMemcpyAsync(b->dws, t.bytes.data(), t.bytes.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        flip_batch_destroy(b);
        return FLIP_E_HIP;
    }
    *out = b;
    return FLIP_OK;
}

flip_status flip_batch_step(flip_batch* b, int nsteps, void* hip_stream)
{
    if (!b || nsteps < 0) return FLIP_E_INVALID;
    hipStream_t st = (hipStream_t)hip_stream;
    flip_status first = FLIP_OK;
    for (int k = 0; k < nsteps; ++k) {
        flip_status r = b->prec == FLIP_FP64 ? batch_step<double>(b, st) : batch_step<float>(b, st);
        if (r == FLIP_E_HIP || r == FLIP_E_STATE) return r;
        if (r != FLIP_OK && first == FLIP_OK) first = r;
    }
    return first;
}

void flip_batch_destroy(flip_batch* b)
{
    if (!b) return;
    // the handles may already be gone: only the batch's own streams are touched
    if (b->last_stream) (void)hipStreamSynchronize(b->last_stream);
    for (hipGraphExec_t* g : {&b->g_pre[0], &b->g_pre[1], &b->g_chunk, &b->g_chunk_small, &b->g_post[0], &b->g_post[1]})
        if (*g) (void)hipGraphExecDestroy(*g);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->h_sum) (void)hipHostFree(b->h_sum);
    delete b;
}

}  // extern "C"
