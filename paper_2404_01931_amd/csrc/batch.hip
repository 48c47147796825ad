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
// Multigrid batches: an iteration launched past convergence costs a dozen
// launches, so they start with the previous step's largest count and then
// test every MG_NEXT_CHUNK iterations (a recorded chunk of that size too).
constexpr int MG_NEXT_CHUNK = 2;

// Host image of the launch tables, uploaded into the batch workspace (once,
// or after each change of a slot batch's scenes).
struct Tables {
    std::vector<char> bytes;
    std::vector<char> live;  // per slot: holds a scene (an empty slot has no workgroups)
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
    uint32_t blocks = 0;  // workgroups of the launch (the scenes' own grids, concatenated)
    uint64_t items = 0;   // work-items of the launch
};

template <typename A>
Site add_site(Tables& t, const std::vector<A>& args, std::vector<uint32_t> blocks, int threads)
{
    std::vector<uint32_t> first(args.size() + 1, 0u);
    uint64_t total = 0;
    for (size_t i = 0; i < args.size(); ++i) {
        if (i < t.live.size() && !t.live[i]) blocks[i] = 0;
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
    Site fill_count, scan_c[3], scatter, tile_flags, scan_t[3], tile_compact, rhs, dir[2], upd[2], project,
        summary;
    PhaseSites ph[2];
    size_t summary_off = 0;  // SolveSummary[ns]
    // multigrid (all scenes or none): levels below the fine grid, deepest scene
    bool mg = false;
    bool fused = false;  // the multigrid update with the fine restriction (FP32 vectors)
    int mg_levels = 0;
    Site mg_types_fine, mg_fine_down, mg_fine_up[2], mg_bottom, upd_down[2];
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
// as the plain step of each handle (capi.hip, run_step). slots[s] is the
// scene of slot s (null: empty; its entries stay zero and it has no
// workgroups); cur0[s] its current particle buffer at an even batch step;
// mg_levels the multigrid levels the launch sequence covers; dws the device
// workspace (null when only sizing).
template <typename T>
void build_sites(const std::vector<flip_handle*>& slots, const std::vector<int>& cur0, int mg_levels,
                 const char* dws, Tables& t, Sites& S)
{
    const size_t ns = slots.size();
    S.fused = S.mg && mg_fused_update(sizeof(T));
    const bool fused = S.fused;
    static flip_handle empty_slot;  // stands in for an empty slot (zero sizes, null pointers)
    std::vector<flip_handle*> hs(ns);
    t.live.assign(ns, 0);
    for (size_t s = 0; s < ns; ++s) {
        hs[s] = slots[s] ? slots[s] : &empty_slot;
        t.live[s] = slots[s] != nullptr;
    }
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
            const int cur = cur0[s] ^ ph, nxt = cur ^ 1;
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
        std::vector<ProjectArgs<T, T>> pr(ns);
        std::vector<uint32_t> bg(ns), bf(ns);
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
            for (int k = 0; k < 2; ++k) {
                // with multigrid the direction kernel reads z = M r from
                // h->mgz, with the fused update that of an odd iteration from
                // h->z (r and z trade places at every update; see enqueue_chunk)
                const T* zdir = (const T*)(S.mg ? (fused && k ? h->z : h->mgz) : h->z);
                DirArgs<T> d{-1, h->tile_nbr, h->diag, zdir, (const T*)h->s[k], (T*)h->s[k ^ 1],
                             fused ? (T*)h->q : nullptr, h->pslots, h->ps};
                UpdArgs<T> u{-1, h->tile_nbr, h->diag, (const T*)h->s[k ^ 1], (T*)h->xin[0], (T*)h->z, h->pslots,
                             h->ps};
                (k ? d1 : d0)[s] = d;
                (k ? u1 : u0)[s] = u;
            }
            const T scale = (T)(c.dt / (c.density * c.dx));
            pr[s] = ProjectArgs<T, T>{h->geo, h->diag, h->tile_slot, (const T*)h->xin[0],
                                      {(const T*)h->f_star[0], (const T*)h->f_star[1], (const T*)h->f_star[2]},
                                      {(T*)h->f_new[0], (T*)h->f_new[1], (T*)h->f_new[2]}, scale};
            bf[s] = (uint32_t)project_blocks(h->geo);
            bg[s] = (uint32_t)h->groups;
        }
        S.rhs = add_site(t, r, bg, TILE_CELLS);
        S.dir[0] = add_site(t, d0, bg, 256);
        S.dir[1] = add_site(t, d1, bg, 256);
        if (!fused) {  // the fused multigrid update has its own sites
            S.upd[0] = add_site(t, u0, bg, 256);
            S.upd[1] = add_site(t, u1, bg, 256);
        }
        S.project = add_site(t, pr, bf, 256);
    }
    if (S.mg) {
        // batched launches run every block of a level (no block lists)
        auto unlisted = [](MgLevel lv) {
            lv.uflag = lv.dlist = lv.ulist = lv.cnt = nullptr;
            return lv;
        };
        const int L = mg_levels;
        S.mg_levels = L;
        std::vector<MgTypesFineArgs> tf(ns);
        std::vector<MgFineArgs<T>> fd(ns), fu0(ns), fu1(ns);
        std::vector<MgPairArgs> bo(ns);
        std::vector<UpdDownArgs<T>> ud0(ns), ud1(ns);
        std::vector<uint32_t> btf(ns), bfine(ns), bbot(ns, 1u);
        for (size_t s = 0; s < ns; ++s) {
            flip_handle* h = hs[s];
            const MgLevel l0 = unlisted(h->mg[0]);
            tf[s] = MgTypesFineArgs{h->geo, h->tile_slot, h->diag, l0};
            btf[s] = (uint32_t)mg_blocks(MG_B_TYPES, l0, l0);
            fd[s] = MgFineArgs<T>{-1, h->geo, h->tile_list, h->tile_nbr, h->diag, (const T*)h->z, l0, nullptr,
                                  nullptr, h->ps};
            // the V-cycle before an even iteration's direction: r in h->z, z
            // to h->mgz; before an odd one the other way round
            fu0[s] = MgFineArgs<T>{-1, h->geo, h->tile_list, h->tile_nbr, h->diag, (const T*)h->z, l0, (T*)h->mgz,
                                   h->pslots, h->ps};
            fu1[s] = fused ? MgFineArgs<T>{-1, h->geo, h->tile_list, h->tile_nbr, h->diag, (const T*)h->mgz, l0,
                                           (T*)h->z, h->pslots, h->ps}
                           : fu0[s];
            bfine[s] = (uint32_t)h->groups;
            for (int k = 0; k < 2; ++k) {
                T* const r = (T*)(k ? h->mgz : h->z);  // r before update k; the new r goes to the other
                T* const r_out = (T*)(k ? h->z : h->mgz);
                (k ? ud1 : ud0)[s] = UpdDownArgs<T>{-1, h->geo, h->tile_list, h->tile_nbr, h->diag,
                                                    (const T*)h->s[k ^ 1], (const T*)h->q, (T*)h->xin[0], r, r_out,
                                                    l0, h->pslots, h->ps};
            }
            const MgLevel bottom = unlisted(h->mg[h->nmg > 0 ? h->nmg - 1 : 0]);
            bo[s] = MgPairArgs{bottom, bottom, h->ps};
        }
        S.mg_types_fine = add_site(t, tf, btf, 256);
        S.mg_fine_down = add_site(t, fd, bfine, 256);
        S.mg_fine_up[0] = add_site(t, fu0, bfine, 256);
        S.mg_fine_up[1] = add_site(t, fu1, bfine, 256);
        S.mg_bottom = add_site(t, bo, bbot, 512);
        if (fused) {
            S.upd_down[0] = add_site(t, ud0, bfine, 256);
            S.upd_down[1] = add_site(t, ud1, bfine, 256);
        }
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
            const int nt = mg_two_sweeps(l) ? MG_BATCH_NT2 : MG_BATCH_NT;
            S.mg_down[l] = add_site(t, a, bd, nt);
            S.mg_up[l] = add_site(t, a, bu, nt);
        }
    }
    {
        // the summary array itself, then the summary launch that fills it
        S.summary_off = t.reserve(sizeof(SolveSummary) * ns);
        SolveSummary* d_sum = dws ? (SolveSummary*)(dws + S.summary_off) : nullptr;
        std::vector<SummaryArgs> a(ns);
        std::vector<uint32_t> b1(ns, 1u);
        for (size_t s = 0; s < ns; ++s) a[s] = SummaryArgs{hs[s]->ps, d_sum ? d_sum + s : nullptr};
        S.summary = add_site(t, a, b1, 64);
    }
}

// every launch site of a step, in a fixed order
template <typename S_, typename F>
void for_each_site(S_& S, F&& f)
{
    f(S.fill_count);
    f(S.scatter);
    f(S.tile_flags);
    f(S.tile_compact);
    f(S.rhs);
    f(S.summary);
    f(S.project);
    for (int i = 0; i < 3; ++i) {
        f(S.scan_c[i]);
        f(S.scan_t[i]);
    }
    for (int k = 0; k < 2; ++k) {
        f(S.dir[k]);
        f(S.upd[k]);
        f(S.ph[k].bin_keys);
        f(S.ph[k].gather);
        f(S.ph[k].p2g);
        f(S.ph[k].g2p);
    }
    if (S.mg) {
        f(S.mg_types_fine);
        f(S.mg_fine_down);
        f(S.mg_fine_up[0]);
        f(S.mg_fine_up[1]);
        f(S.mg_bottom);
        f(S.upd_down[0]);
        f(S.upd_down[1]);
        for (int l = 0; l + 1 < S.mg_levels; ++l) {
            f(S.mg_types[l]);
            f(S.mg_down[l]);
            f(S.mg_up[l]);
        }
    }
}

bool sites_fit(const Sites& S)
{
    auto ok = [](const Site& s) { return s.items < 0xFFFFFFFFull; };
    bool r = ok(S.fill_count) && ok(S.scatter) && ok(S.tile_flags) && ok(S.tile_compact) && ok(S.rhs) &&
             ok(S.summary);
    r = r && ok(S.project);
    for (int i = 0; i < 3; ++i) r = r && ok(S.scan_c[i]) && ok(S.scan_t[i]);
    for (int k = 0; k < 2; ++k)
        r = r && ok(S.dir[k]) && ok(S.upd[k]) && ok(S.ph[k].bin_keys) && ok(S.ph[k].gather) && ok(S.ph[k].p2g) &&
            ok(S.ph[k].g2p);
    if (S.mg) {
        r = r && ok(S.mg_types_fine) && ok(S.mg_fine_down) && ok(S.mg_fine_up[0]) && ok(S.mg_fine_up[1]) &&
            ok(S.mg_bottom) &&
            ok(S.upd_down[0]) && ok(S.upd_down[1]);
        for (int l = 0; l + 1 < S.mg_levels; ++l) r = r && ok(S.mg_types[l]) && ok(S.mg_down[l]) && ok(S.mg_up[l]);
    }
    return r;
}

// a handle a batch of this precision and preconditioner can step
flip_status check_handle(const flip_handle* h, int prec, bool mg)
{
    if (!h) return FLIP_E_INVALID;
    if (h->prec != FLIP_FP32 && h->prec != FLIP_FP64) return FLIP_E_INVALID;
    if (h->prec != prec) return FLIP_E_INVALID;
    if (h->cfg.flags & (FLIP_FLAG_NO_PROJECTION | FLIP_FLAG_KERNEL_TIMING | FLIP_FLAG_DIAGNOSTICS |
                        FLIP_FLAG_RED_BLACK_GS | FLIP_FLAG_ADAPTIVE_DT | FLIP_FLAG_RESEED))
        return FLIP_E_INVALID;
    // the preconditioner is the same for every scene of a batch
    if (((h->cfg.flags & FLIP_FLAG_MULTIGRID) != 0) != mg) return FLIP_E_INVALID;
    return FLIP_OK;
}

flip_status check_handles(flip_handle* const* handles, int nscenes, int* prec, bool* mg)
{
    if (!handles || nscenes < 1 || nscenes > FLIP_BATCH_MAX_SCENES) return FLIP_E_INVALID;
    if (!handles[0]) return FLIP_E_INVALID;
    *prec = handles[0]->prec;
    *mg = (handles[0]->cfg.flags & FLIP_FLAG_MULTIGRID) != 0;
    for (int s = 0; s < nscenes; ++s) {
        flip_status v = check_handle(handles[s], *prec, *mg);
        if (v != FLIP_OK) return v;
        for (int q = 0; q < s; ++q)
            if (handles[q] == handles[s]) return FLIP_E_INVALID;
    }
    return FLIP_OK;
}

// multigrid levels of a grid (each axis halved, ceil, until none exceeds the bottom side)
int mg_levels_of(int nx, int ny, int nz)
{
    int l = 0;
    do {
        nx = (nx + 1) / 2;
        ny = (ny + 1) / 2;
        nz = (nz + 1) / 2;
        ++l;
    } while ((nx > MG_BOTTOM_SIDE || ny > MG_BOTTOM_SIDE || nz > MG_BOTTOM_SIDE) && l < MG_MAX_LEVELS);
    return l;
}

flip_status build_tables(const std::vector<flip_handle*>& slots, const std::vector<int>& cur0, int prec, bool mg,
                         int mg_levels, const char* dws, Tables& t, Sites& S)
{
    S.mg = mg;
    if (prec == FLIP_FP64)
        build_sites<double>(slots, cur0, mg_levels, dws, t, S);
    else
        build_sites<float>(slots, cur0, mg_levels, dws, t, S);
    return sites_fit(S) ? FLIP_OK : FLIP_E_INVALID;
}

// A recorded graph keeps the grid each launch had when it was recorded, and
// its workgroups loop over however many workgroups the scenes present need, so
// it stays correct whatever the scenes; it is recorded again only when a
// launch needs more than twice the workgroups it was recorded with (or had
// none), or a quarter of them or fewer (idle workgroups).
bool grids_drifted(const Sites& cur, const Sites& rec)
{
    std::vector<uint32_t> a, r;
    for_each_site(cur, [&](const Site& x) { a.push_back(x.blocks); });
    for_each_site(rec, [&](const Site& x) { r.push_back(std::max<uint32_t>(x.blocks, 1u)); });
    if (a.size() != r.size()) return true;
    for (size_t i = 0; i < a.size(); ++i) {
        if (a[i] > 2ull * r[i]) return true;
        if (a[i] > 0 && 4ull * a[i] <= r[i]) return true;
    }
    return false;
}

}  // namespace

struct flip_batch {
    std::vector<flip_handle*> slot;  // scene of each slot (null: empty)
    std::vector<int> cur0;           // per slot: the scene's current particle buffer at an even step
    int prec = FLIP_FP32;
    bool mg = false;
    int mg_levels = 0;               // levels the launch sequence covers
    uint32_t flags = 0;
    bool slots_api = false;          // made by flip_batch_create_slots (fixed grids, attach / detach)
    int max_dims[3] = {0, 0, 0};     // largest grid a slot batch takes
    char* dws = nullptr;
    size_t table_bytes = 0;
    Sites S;
    Sites S_rec;                     // the launch grids the graphs were recorded with
    char* h_table = nullptr;         // pinned image of the tables
    bool dirty = true;               // the scenes changed since the tables were uploaded
    SolveSummary* h_sum = nullptr;   // pinned host copy of the summaries
    int phase = 0;                   // steps taken, mod 2
    int64_t steps = 0;
    hipStream_t cap_stream = nullptr;
    hipStream_t last_stream = nullptr;  // stream of the last step
    hipGraphExec_t g_pre[2] = {nullptr, nullptr};
    hipGraphExec_t g_chunk = nullptr;
    hipGraphExec_t g_chunk_small = nullptr;  // MG_NEXT_CHUNK iterations (multigrid batches)
    hipGraphExec_t g_post[2] = {nullptr, nullptr};
    flip_batch_info info{};
};

namespace {

// A slot batch launches every site, at least one workgroup: a recorded graph
// then holds every launch, whatever the scenes at recording time (a launch
// whose scenes need no workgroup exits at once).
BatchLaunch L(const flip_batch* b, const Site& s)
{
    BatchLaunch l;
    l.args = b->dws + s.args_off;
    l.first = (const uint32_t*)(b->dws + s.first_off);
    l.ns = s.ns;
    l.blocks = b->slots_api ? std::max<uint32_t>(s.blocks, 1u) : s.blocks;
    return l;
}

// one multigrid V-cycle z = M r of every scene: the restrictions level by
// level down to the deepest scene's coarsest level, every scene's coarsest
// sweeps, then the prolongations back up (a scene takes part in the level
// launches it has, so its own order is down, bottom, up)
// (fine_down false: the fine level's down kernel ran inside the update;
// parity: that of the direction kernel that follows, which sets where r and
// z are)
template <typename T>
void enqueue_vcycle(const flip_batch* b, hipStream_t st, bool fine_down, int parity)
{
    const Sites& S = b->S;
    if (fine_down) launch_b_mg_fine<T>(false, L(b, S.mg_fine_down), st);
    for (int l = 0; l + 1 < S.mg_levels; ++l)
        launch_b_mg_level<T>(MG_B_DOWN, mg_two_sweeps(l), L(b, S.mg_down[l]), st);
    launch_b_mg_level<T>(MG_B_BOTTOM, false, L(b, S.mg_bottom), st);
    for (int l = S.mg_levels - 2; l >= 0; --l) launch_b_mg_level<T>(MG_B_UP, mg_two_sweeps(l), L(b, S.mg_up[l]), st);
    launch_b_mg_fine<T>(true, L(b, S.mg_fine_up[parity]), st);
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
        enqueue_vcycle<T>(b, st, true, 0);
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
        if (S.fused) {
            launch_b_pcg_update_down<T>(L(b, S.upd_down[i & 1]), st);
            enqueue_vcycle<T>(b, st, false, (i + 1) & 1);
        } else {
            launch_b_pcg_update<T>(S.mg, L(b, S.upd[i & 1]), st);
            if (S.mg) enqueue_vcycle<T>(b, st, true, (i + 1) & 1);
        }
        launch_b_pcg_direction<T>(L(b, S.dir[(i + 1) & 1]), st);
    }
    launch_b_summary(L(b, S.summary), st);
}

template <typename T>
void enqueue_post(const flip_batch* b, int ph, hipStream_t st)
{
    const Sites& S = b->S;
    launch_b_project3<T, T>(L(b, S.project), st);
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
    b->info.graph_captures += 1;
    return hipGetLastError() == hipSuccess ? FLIP_OK : FLIP_E_HIP;
}

flip_status launch_graph(flip_batch* b, hipGraphExec_t g, hipStream_t st)
{
    HIP_TRY(hipGraphLaunch(g, st));
    b->info.graph_launches += 1;
    return FLIP_OK;
}

// rebuild the tables for the current scenes and upload them (stream-ordered
// before the step's launches)
flip_status upload_tables(flip_batch* b, hipStream_t st)
{
    Tables t;
    Sites S;
    flip_status v = build_tables(b->slot, b->cur0, b->prec, b->mg, b->mg_levels, b->dws, t, S);
    if (v != FLIP_OK) return v;
    if (t.bytes.size() != b->table_bytes) return FLIP_E_STATE;  // the layout is fixed by the slot count
    // the previous upload has completed: every step ends with a synchronised summary read
    std::memcpy(b->h_table, t.bytes.data(), t.bytes.size());
    HIP_TRY(hipMemcpyAsync(b->dws, b->h_table, t.bytes.size(), hipMemcpyHostToDevice, st));
    b->S = S;
    b->dirty = false;
    b->info.table_uploads += 1;
    return FLIP_OK;
}

void drop_graphs(flip_batch* b)
{
    for (hipGraphExec_t* g : {&b->g_pre[0], &b->g_pre[1], &b->g_chunk, &b->g_chunk_small, &b->g_post[0], &b->g_post[1]})
        if (*g) {
            (void)hipGraphExecDestroy(*g);
            *g = nullptr;
        }
}

template <typename T>
flip_status batch_step(flip_batch* b, hipStream_t st)
{
    const int ns = (int)b->slot.size();
    const int ph = b->phase;
    b->last_stream = st;
    bool any = false;
    for (int s = 0; s < ns; ++s) {
        const flip_handle* h = b->slot[s];
        if (!h) continue;
        any = true;
        if (h->cur != (b->cur0[s] ^ ph)) return FLIP_E_STATE;  // stepped outside the batch
    }
    if (!any) return FLIP_OK;  // an empty slot batch: nothing to step
    if (b->dirty) {
        flip_status v = upload_tables(b, st);
        if (v != FLIP_OK) return v;
        // record the graphs again when launches outgrew the grids they were
        // recorded with, or shrank far below them
        if (b->g_chunk && grids_drifted(b->S, b->S_rec)) {
            HIP_TRY(hipStreamSynchronize(st));  // no replay of the old graphs is still running
            drop_graphs(b);
        }
    }
    const bool graphs = (b->flags & FLIP_BATCH_GRAPHS) && b->steps >= 1;
    if (graphs) {
        const bool any = b->g_pre[0] || b->g_pre[1] || b->g_chunk || b->g_post[0] || b->g_post[1];
        if (!any) b->S_rec = b->S;  // a new set of graphs: recorded with the current grids
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
        flip_status r = launch_graph(b, b->g_pre[ph], st);
        if (r != FLIP_OK) return r;
    } else {
        enqueue_pre<T>(b, ph, st);
    }

    // the solve: chunks of iterations until no scene is running
    int prev = 0, max_cap = 0;
    for (const flip_handle* h : b->slot)
        if (h) {
            prev = std::max(prev, h->prev_iters);
            max_cap = std::max(max_cap, solve_iter_cap(h->cfg));
        }
    const bool mg = b->S.mg;
    int chunk = prev > 2 ? (mg ? prev : prev - 2) : FIRST_CHUNK;
    const int unit = graphs && !mg ? GRAPH_CHUNK : 2;
    chunk = (chunk + unit - 1) / unit * unit;
    int launched = 0;
    const size_t sum_bytes = sizeof(SolveSummary) * ns;
    for (;;) {
        if (graphs) {
            for (int q = 0; q < chunk / GRAPH_CHUNK; ++q) {
                flip_status r = launch_graph(b, b->g_chunk, st);
                if (r != FLIP_OK) return r;
            }
            for (int q = 0; q < (chunk % GRAPH_CHUNK) / MG_NEXT_CHUNK; ++q) {
                flip_status r = launch_graph(b, b->g_chunk_small, st);
                if (r != FLIP_OK) return r;
            }
        } else {
            enqueue_chunk<T>(b, chunk, st);
        }
        launched += chunk;
        HIP_TRY(hipMemcpyAsync(b->h_sum, b->dws + b->S.summary_off, sum_bytes, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        bool running = false;
        for (int s = 0; s < ns; ++s) running = running || (b->slot[s] && b->h_sum[s].done == PCG_RUNNING);
        if (!running || launched > max_cap + 8) break;
        chunk = mg ? MG_NEXT_CHUNK : (graphs ? GRAPH_CHUNK : NEXT_CHUNK);
    }

    if (graphs) {
        flip_status r = launch_graph(b, b->g_post[ph], st);
        if (r != FLIP_OK) return r;
    } else {
        enqueue_post<T>(b, ph, st);
    }
    if (hipGetLastError() != hipSuccess) return FLIP_E_HIP;

    flip_status first = FLIP_OK;
    for (int s = 0; s < ns; ++s) {
        flip_handle* h = b->slot[s];
        if (!h) continue;
        const SolveSummary& q = b->h_sum[s];
        flip_status ret = FLIP_OK;
        if (q.done == PCG_MAX_ITERS || q.done == PCG_RUNNING) ret = FLIP_E_NOT_CONVERGED;
        if (q.done == PCG_BREAKDOWN) ret = q.sync_error ? FLIP_E_HIP : FLIP_E_NONFINITE;
        const int status = q.done == PCG_CONVERGED ? 0 : (q.done == PCG_BREAKDOWN ? 2 : 1);
        record_step(h, q.n_active > 0, status, q.n_active, q.nfluid, q.max_b, q.max_r, q.iter, 0, ret);
        h->prev_iters = q.iter;
        h->keys_ready = false;  // a batched step does not bin the positions it writes
        h->cur ^= 1;
        h->scur = (q.iter & 1);
        h->xi = 0;
        h->last_stream = st;
        if (ret != FLIP_OK && first == FLIP_OK) first = ret;
    }
    b->phase ^= 1;
    b->steps += 1;
    b->info.steps += 1;
    return first;
}

// a batch object with its tables sized for `slots` (the entries filled by build_tables)
flip_status new_batch(const std::vector<flip_handle*>& slots, int prec, bool mg, int mg_levels, uint32_t flags,
                      bool slots_api, void* d_ws, size_t ws_bytes, flip_batch** out)
{
    flip_batch* b = new (std::nothrow) flip_batch();
    if (!b) return FLIP_E_INVALID;
    b->slot = slots;
    b->cur0.assign(slots.size(), 0);
    for (size_t s = 0; s < slots.size(); ++s)
        if (slots[s]) b->cur0[s] = slots[s]->cur;
    b->prec = prec;
    b->mg = mg;
    b->mg_levels = mg_levels;
    b->flags = flags;
    b->slots_api = slots_api;
    Tables t;
    Sites S;
    flip_status v = build_tables(b->slot, b->cur0, prec, mg, mg_levels, nullptr, t, S);
    if (v != FLIP_OK) {
        delete b;
        return v;
    }
    if (!d_ws || ws_bytes < t.bytes.size() || ((uintptr_t)d_ws & (TABLE_ALIGN - 1))) {
        delete b;
        return FLIP_E_WORKSPACE;
    }
    b->dws = (char*)d_ws;
    b->table_bytes = t.bytes.size();
    b->S = S;
    b->info.nslots = (int)slots.size();
    if (hipHostMalloc((void**)&b->h_sum, sizeof(SolveSummary) * slots.size(), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->h_table, b->table_bytes, hipHostMallocDefault) != hipSuccess) {
        flip_batch_destroy(b);
        return FLIP_E_HIP;
    }
    *out = b;
    return FLIP_OK;
}

bool slot_batch_takes(const flip_batch* b, const flip_handle* h)
{
    return h->cfg.nx <= b->max_dims[0] && h->cfg.ny <= b->max_dims[1] && h->cfg.nz <= b->max_dims[2] &&
           h->nmg <= b->mg_levels;
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
    std::vector<int> cur0(nscenes, 0);
    int levels = 0;
    for (flip_handle* h : hs) levels = std::max(levels, h->nmg);
    Tables t;
    Sites S;
    v = build_tables(hs, cur0, prec, mg, levels, nullptr, t, S);
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
    std::vector<flip_handle*> hs(handles, handles + nscenes);
    int levels = 0;
    for (flip_handle* h : hs) levels = std::max(levels, h->nmg);
    flip_batch* b = nullptr;
    v = new_batch(hs, prec, mg, levels, flags, false, d_ws, ws_bytes, &b);
    if (v != FLIP_OK) return v;
    for (flip_handle* h : hs) {
        b->max_dims[0] = std::max(b->max_dims[0], h->cfg.nx);
        b->max_dims[1] = std::max(b->max_dims[1], h->cfg.ny);
        b->max_dims[2] = std::max(b->max_dims[2], h->cfg.nz);
    }
    b->info.occupied = nscenes;
    hipStream_t st = (hipStream_t)hip_stream;
    if (upload_tables(b, st) != FLIP_OK || hipStreamSynchronize(st) != hipSuccess) {
        flip_batch_destroy(b);
        return FLIP_E_HIP;
    }
    *out = b;
    return FLIP_OK;
}

flip_status flip_batch_slots_workspace_bytes(const flip_batch_slots* spec, size_t* out_bytes)
{
    if (!spec || !out_bytes) return FLIP_E_INVALID;
    if (spec->nslots < 1 || spec->nslots > FLIP_BATCH_MAX_SCENES) return FLIP_E_INVALID;
    if (spec->precision != FLIP_FP32 && spec->precision != FLIP_FP64) return FLIP_E_INVALID;
    if (spec->max_nx < 1 || spec->max_ny < 1 || spec->max_nz < 1) return FLIP_E_INVALID;
    std::vector<flip_handle*> hs(spec->nslots, nullptr);
    std::vector<int> cur0(spec->nslots, 0);
    const bool mg = (spec->flags & FLIP_BATCH_MULTIGRID) != 0;
    Tables t;
    Sites S;
    flip_status v = build_tables(hs, cur0, spec->precision, mg, mg ? mg_levels_of(spec->max_nx, spec->max_ny, spec->max_nz) : 0,
                                 nullptr, t, S);
    if (v != FLIP_OK) return v;
    *out_bytes = t.bytes.size();
    return FLIP_OK;
}

flip_status flip_batch_create_slots(const flip_batch_slots* spec, void* d_ws, size_t ws_bytes, void* hip_stream,
                                    flip_batch** out)
{
    if (!out) return FLIP_E_INVALID;
    *out = nullptr;
    size_t need = 0;
    flip_status v = flip_batch_slots_workspace_bytes(spec, &need);
    if (v != FLIP_OK) return v;
    if (spec->flags & ~(uint32_t)(FLIP_BATCH_GRAPHS | FLIP_BATCH_MULTIGRID)) return FLIP_E_INVALID;
    const bool mg = (spec->flags & FLIP_BATCH_MULTIGRID) != 0;
    std::vector<flip_handle*> hs(spec->nslots, nullptr);
    flip_batch* b = nullptr;
    v = new_batch(hs, spec->precision, mg, mg ? mg_levels_of(spec->max_nx, spec->max_ny, spec->max_nz) : 0,
                  spec->flags & FLIP_BATCH_GRAPHS, true, d_ws, ws_bytes, &b);
    if (v != FLIP_OK) return v;
    b->max_dims[0] = spec->max_nx;
    b->max_dims[1] = spec->max_ny;
    b->max_dims[2] = spec->max_nz;
    b->last_stream = (hipStream_t)hip_stream;
    *out = b;
    return FLIP_OK;
}

flip_status flip_batch_attach(flip_batch* b, int slot, flip_handle* h)
{
    if (!b || !h || !b->slots_api) return FLIP_E_INVALID;
    if (slot < 0 || slot >= (int)b->slot.size() || b->slot[slot]) return FLIP_E_INVALID;
    flip_status v = check_handle(h, b->prec, b->mg);
    if (v != FLIP_OK) return v;
    if (!slot_batch_takes(b, h)) return FLIP_E_INVALID;
    for (const flip_handle* o : b->slot)
        if (o == h) return FLIP_E_INVALID;
    b->slot[slot] = h;
    b->cur0[slot] = h->cur ^ b->phase;
    b->dirty = true;
    b->info.occupied += 1;
    return FLIP_OK;
}

flip_status flip_batch_detach(flip_batch* b, int slot)
{
    if (!b || !b->slots_api) return FLIP_E_INVALID;
    if (slot < 0 || slot >= (int)b->slot.size() || !b->slot[slot]) return FLIP_E_INVALID;
    b->slot[slot] = nullptr;
    b->dirty = true;
    b->info.occupied -= 1;
    return FLIP_OK;
}

flip_status flip_batch_get_info(const flip_batch* b, flip_batch_info* out)
{
    if (!b || !out) return FLIP_E_INVALID;
    *out = b->info;
    return FLIP_OK;
}

flip_status flip_batch_step(flip_batch* b, int nsteps, void* hip_stream)
{
    if (!b || nsteps < 0) return FLIP_E_INVALID;
    hipStream_t st = (hipStream_t)hip_stream;
    flip_status first = FLIP_OK;
    for (int k = 0; k < nsteps; ++k) {
        flip_status r = b->prec == FLIP_FP64 ? batch_step<double>(b, st) : batch_step<float>(b, st);
        if (r == FLIP_E_HIP || r == FLIP_E_STATE || r == FLIP_E_INVALID) return r;
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
    if (b->h_table) (void)hipHostFree(b->h_table);
    delete b;
}

}  // extern "C"
