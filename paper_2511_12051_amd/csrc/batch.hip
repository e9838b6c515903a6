// Batched runs of the whole path over independent mini-stacks, one persistent
// launch per stage and kernel variant, captured once into a HIP graph and
// replayed (host side; the kernels' batched wrappers live with each stage).
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "batch_device.hpp"
#include "internal.hpp"

using namespace plk;

namespace {

template <typename Args>
struct Group {
    std::vector<int> members;     // item indices
    std::vector<Args> args;       // per member
    std::vector<int64_t> starts;  // members + 1 block offsets
    Args* d_args = nullptr;
    int64_t* d_starts = nullptr;
    int variant = 0;    // stats: 16-byte loads; coherence: tile; linking: (N + 3) / 4
    int threads = 0;
    size_t lds = 0;
    int64_t grid = 0;
    int mult = 4;       // persistent grid = mult x (resident workgroups per CU) x CUs; 0: one per block
    int txo = 16, rows = 0;  // coherence tile
    float best_ms = -1.f;

    bool empty() const { return members.empty(); }
    int64_t total() const { return starts.empty() ? 0 : starts.back(); }
    BatchRange<Args> range() const { return BatchRange<Args>{d_args, d_starts, (int)args.size(), total()}; }
};

template <typename Args>
void add_member(Group<Args>& g, int item, const Args& a, int64_t blocks) {
    if (g.starts.empty()) g.starts.push_back(0);
    g.members.push_back(item);
    g.args.push_back(a);
    g.starts.push_back(g.starts.back() + blocks);
}

template <typename Args>
pl_status upload(Group<Args>& g) {
    if (g.empty()) return PL_OK;
    if (!g.d_args) {
        pl_status st = hip_ok(hipMalloc(&g.d_args, sizeof(Args) * g.args.size()), "pl_batch_plan: item table");
        if (st != PL_OK) return st;
        st = hip_ok(hipMalloc(&g.d_starts, sizeof(int64_t) * g.starts.size()), "pl_batch_plan: item table");
        if (st != PL_OK) return st;
    }
    pl_status st = hip_ok(hipMemcpy(g.d_args, g.args.data(), sizeof(Args) * g.args.size(), hipMemcpyHostToDevice),
                          "pl_batch_plan: item table upload");
    if (st != PL_OK) return st;
    return hip_ok(hipMemcpy(g.d_starts, g.starts.data(), sizeof(int64_t) * g.starts.size(), hipMemcpyHostToDevice),
                  "pl_batch_plan: item table upload");
}

template <typename Args>
void release(Group<Args>& g) {
    if (g.d_args) (void)hipFree(g.d_args);
    if (g.d_starts) (void)hipFree(g.d_starts);
    g.d_args = nullptr;
    g.d_starts = nullptr;
}

}  // namespace

namespace {

// the launches of one level: one group per stage and kernel variant
struct Level {
    Group<StatsArgs> stats[2];   // [0] plain loads, [1] 16-byte loads
    Group<GlrtArgs> glrt;
    Group<CohArgs> coh[2];       // [0] 16-row tile, [1] 32-row tile
    Group<LinkArgs> link[9];     // by (N + 3) / 4
    Group<CompressArgs> comp;
};

}  // namespace

// per-item arguments of every stage, kept for the single-launch form
struct ItemArgs {
    bool has_stats = false, stats_vec = false, has_comp = false;
    StatsArgs stats{};
    int64_t stats_blocks = 0;
    GlrtArgs glrt{};
    int64_t glrt_blocks = 0;
    size_t glrt_lds = 0;
    CohArgs coh{};
    LinkArgs link{};
    int64_t link_blocks = 0;
    CompressArgs comp{};
    int64_t comp_blocks = 0;
};

struct pl_batch {
    std::vector<pl_batch_item> items;
    std::vector<ItemArgs> iargs;
    // single-launch form: the whole run as one persistent kernel
    bool single = false, single_ok = false;
    std::string single_why;
    void* mega_mem = nullptr;
    MegaPlan mega{};
    int mega_nseg = 0;
    size_t mega_lds = 0;
    int64_t mega_grid = 0;
    float mega_ms = -1.f, graph_ms = -1.f;
    std::vector<void*> allocations;
    std::vector<int> level_ids;  // distinct levels, increasing
    std::vector<Level> levels;
    bool split = false;
    int cus = 1;
    hipStream_t own = nullptr;   // capture / replay stream (default priority)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int runs = 0;
};

namespace {

// persistent grid of a group: resident workgroups per CU x CUs x mult,
// never more than the group's blocks
template <typename Args>
pl_status size_grid(const pl_batch* b, Group<Args>& g, const void* fn) {
    if (g.empty()) return PL_OK;
    const int64_t total = g.total();
    if (g.mult <= 0) {
        g.grid = total;
    } else {
        int per_cu = 0;
        pl_status st = hip_ok(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, g.threads, g.lds),
                              "pl_batch_plan: occupancy query");
        if (st != PL_OK) return st;
        if (per_cu < 1) per_cu = 1;
        g.grid = (int64_t)per_cu * b->cus * g.mult;
    }
    if (g.grid > total) g.grid = total;
    if (g.grid < 1) g.grid = 1;
    if (g.grid > 2147483647LL) g.grid = 2147483647LL;
    return PL_OK;
}

pl_status configure_coherence(pl_batch* b, Level& L, int v, int txo, int rows) {
    Group<CohArgs>& g = L.coh[v];
    g.starts.assign(1, 0);
    g.lds = 0;
    for (size_t m = 0; m < g.members.size(); ++m) {
        int64_t blocks = 0;
        const size_t lds = coherence_args(&g.args[m], g.variant, b->split, txo, rows, &blocks);
        if (!lds) return fail(PL_ERR_UNSUPPORTED, "pl_batch_plan: window too large for the coherence tile");
        if (lds > g.lds) g.lds = lds;
        g.starts.push_back(g.starts.back() + blocks);
    }
    g.txo = txo;
    g.rows = rows;
    pl_status st = allow_dynamic_lds(coherence_batch_fn(g.variant, b->split), g.lds);
    if (st != PL_OK) return st;
    st = size_grid(b, g, coherence_batch_fn(g.variant, b->split));
    if (st != PL_OK) return st;
    return upload(g);
}

pl_status enqueue_front(pl_batch* b, Level& L, hipStream_t s) {  // statistics and GLRT
    for (int v = 0; v < 2; ++v) {
        if (L.stats[v].empty()) continue;
        pl_status st = launch_amp_stats_batch(L.stats[v].range(), v == 1, L.stats[v].grid, s);
        if (st != PL_OK) return st;
    }
    return launch_shp_select_batch(L.glrt.range(), L.glrt.threads, L.glrt.lds, L.glrt.grid, s);
}

pl_status enqueue_coherence(pl_batch* b, Level& L, hipStream_t s) {
    for (int v = 0; v < 2; ++v) {
        if (L.coh[v].empty()) continue;
        pl_status st = launch_coherence_batch(L.coh[v].range(), L.coh[v].variant, b->split, L.coh[v].lds,
                                              L.coh[v].grid, s);
        if (st != PL_OK) return st;
    }
    return PL_OK;
}

pl_status enqueue_link(Level& L, hipStream_t s) {
    for (auto& g : L.link) {
        if (g.empty()) continue;
        pl_status st = launch_phase_link_batch(g.range(), g.variant, g.grid, s);
        if (st != PL_OK) return st;
    }
    return PL_OK;
}

pl_status enqueue_level(pl_batch* b, Level& L, hipStream_t s) {
    pl_status st = enqueue_front(b, L, s);
    if (st == PL_OK) st = enqueue_coherence(b, L, s);
    if (st == PL_OK) st = enqueue_link(L, s);
    if (st == PL_OK && !L.comp.empty()) st = launch_compress_batch(L.comp.range(), L.comp.grid, s);
    return st;
}

pl_status enqueue_all(pl_batch* b, hipStream_t s) {
    if (b->single) return launch_mega(b->mega, b->split, b->mega_lds, b->mega_grid, s);
    for (auto& L : b->levels) {
        pl_status st = enqueue_level(b, L, s);
        if (st != PL_OK) return st;
    }
    return PL_OK;
}

// average device time of fn over reps launches after one warm-up
template <typename F>
pl_status time_ms(hipStream_t s, F fn, int reps, float* ms) {
    hipEvent_t e0, e1;
    pl_status st = hip_ok(hipEventCreate(&e0), "pl_batch_plan: event");
    if (st != PL_OK) return st;
    st = hip_ok(hipEventCreate(&e1), "pl_batch_plan: event");
    if (st != PL_OK) {
        (void)hipEventDestroy(e0);
        return st;
    }
    st = fn();
    if (st == PL_OK) st = hip_ok(hipEventRecord(e0, s), "pl_batch_plan: event");
    for (int r = 0; r < reps && st == PL_OK; ++r) st = fn();
    if (st == PL_OK) st = hip_ok(hipEventRecord(e1, s), "pl_batch_plan: event");
    if (st == PL_OK) st = hip_ok(hipEventSynchronize(e1), "pl_batch_plan: autotune run");
    if (st == PL_OK) st = hip_ok(hipEventElapsedTime(ms, e0, e1), "pl_batch_plan: event");
    *ms /= (float)reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

// Level by level (a level's inputs may be the compressed SLCs of earlier
// ones): time the candidate coherence tiles and linking grids, keep the
// fastest, then run the level so that the next one sees its outputs.
pl_status autotune(pl_batch* b) {
    hipStream_t s = b->own;
    static const int tiles[][2] = {{16, 0}, {12, 0}, {8, 0}, {16, 2}, {12, 8}, {4, 0}};
    for (auto& L : b->levels) {
        pl_status st = enqueue_front(b, L, s);  // SHP masks of the current inputs
        if (st != PL_OK) return st;
        for (int v = 0; v < 2; ++v) {
            Group<CohArgs>& g = L.coh[v];
            if (g.empty()) continue;
            float best = 0.f;
            int bt = coherence_strip(g.variant), br = 0, bm = 4;
            for (int mult : {4, 0}) {
                for (auto& t : tiles) {
                    g.mult = mult;
                    st = configure_coherence(b, L, v, t[0], t[1]);
                    if (st != PL_OK) return st;
                    float ms = 0.f;
                    st = time_ms(s, [&] { return launch_coherence_batch(g.range(), g.variant, b->split, g.lds, g.grid, s); },
                                 2, &ms);
                    if (st != PL_OK) return st;
                    if (best == 0.f || ms < best) {
                        best = ms;
                        bt = t[0];
                        br = t[1];
                        bm = mult;
                    }
                }
            }
            g.mult = bm;
            st = configure_coherence(b, L, v, bt, br);
            if (st != PL_OK) return st;
            g.best_ms = best;
        }
        st = enqueue_coherence(b, L, s);  // coherence of the current inputs for the linking runs
        if (st != PL_OK) return st;
        for (auto& g : L.link) {
            if (g.empty()) continue;
            float best = 0.f;
            int bm = g.mult;
            for (int mult : {1, 2, 4, 0}) {
                g.mult = mult;
                st = size_grid(b, g, phase_link_batch_fn(g.variant));
                if (st != PL_OK) return st;
                float ms = 0.f;
                st = time_ms(s, [&] { return launch_phase_link_batch(g.range(), g.variant, g.grid, s); }, 2, &ms);
                if (st != PL_OK) return st;
                if (best == 0.f || ms < best) {
                    best = ms;
                    bm = mult;
                }
            }
            g.mult = bm;
            st = size_grid(b, g, phase_link_batch_fn(g.variant));
            if (st != PL_OK) return st;
            g.best_ms = best;
        }
        if (!L.comp.empty()) {
            st = launch_compress_batch(L.comp.range(), L.comp.grid, s);
            if (st != PL_OK) return st;
        }
    }
    return hip_ok(hipStreamSynchronize(s), "pl_batch_plan: autotune");
}

// The single-launch plan: one segment per (item, stage), queued in an order
// that respects every dependency, each with the segments it waits for.  Leaves
// single_ok false (with the reason) when some item does not fit the 512-thread
// workgroup or the LDS of one workgroup.
constexpr int kMegaStatsPerUnit = 64, kMegaLinkPerUnit = 16, kMegaCompressPerUnit = 64;

pl_status build_mega(pl_batch* b) {
    const int n = (int)b->items.size();
    std::vector<MegaSeg> seg;
    std::vector<StatsArgs> st;
    std::vector<GlrtArgs> gl;
    std::vector<CohArgs> co;
    std::vector<LinkArgs> li;
    std::vector<CompressArgs> cp;
    std::vector<int> s_stats(n, -1), s_glrt(n, -1), s_coh(n, -1), s_link(n, -1), s_comp(n, -1);
    size_t lds = 0;
    auto reject = [&](const char* why) {
        b->single_ok = false;
        b->single_why = why;
        return PL_OK;
    };
    auto add = [&](int stage, int arg, int64_t blocks, int per_unit, const std::vector<int>& deps) {
        MegaSeg m{};
        m.stage = stage;
        m.arg = arg;
        m.blocks = blocks;
        m.per_unit = per_unit;
        m.units = (blocks + per_unit - 1) / per_unit;
        m.ndep = 0;
        for (int d : deps)
            if (d >= 0) m.dep[m.ndep++] = d;
        seg.push_back(m);
        return (int)seg.size() - 1;
    };
    // Queue order: statistics and GLRT of the first level; then per level its
    // coherence, the next level's statistics and GLRT (which depend on
    // nothing of this level, so they fill the wait for this level's
    // coherence to drain), linking and compression.
    std::vector<std::pair<int, int>> order;  // (level index, stage)
    const int nl = (int)b->level_ids.size();
    order.push_back({0, 0});
    order.push_back({0, 1});
    for (int l = 0; l < nl; ++l) {
        order.push_back({l, 2});
        if (l + 1 < nl) {
            order.push_back({l + 1, 0});
            order.push_back({l + 1, 1});
        }
        order.push_back({l, 3});
        order.push_back({l, 4});
    }
    for (const auto& [level_index, stage] : order) {
        const int lvl = b->level_ids[level_index];
        {
            for (int k = 0; k < n; ++k) {
                if (b->items[k].level != lvl) continue;
                const ItemArgs& A = b->iargs[k];
                if (stage == 0 && A.has_stats) {
                    st.push_back(A.stats);
                    s_stats[k] = add(A.stats_vec ? MS_STATS_VEC : MS_STATS_SCALAR, (int)st.size() - 1, A.stats_blocks,
                                     kMegaStatsPerUnit, {});
                } else if (stage == 1) {
                    if (A.glrt.TX * A.glrt.TY > mega_threads() / 2)
                        return reject("GLRT tile larger than half the workgroup");
                    if (2 * A.glrt_lds > lds) lds = 2 * A.glrt_lds;  // one tile per half
                    gl.push_back(A.glrt);
                    s_glrt[k] = add(MS_GLRT, (int)gl.size() - 1, A.glrt_blocks, 2, {s_stats[k]});  // a tile per half
                } else if (stage == 2) {
                    CohArgs a = A.coh;
                    const int nt = a.N <= 16 ? 16 : 32;
                    int64_t blocks = 0;
                    const size_t cl = coherence_args(&a, nt, b->split, mega_threads() / 64, 0, &blocks);
                    if (!cl) return reject("coherence tile does not fit in LDS");
                    if ((int64_t)a.N * (a.tile_w >> 1) > (int64_t)8 * mega_threads())
                        return reject("coherence rows too wide for the workgroup's staging");
                    if (cl > lds) lds = cl;
                    co.push_back(a);
                    std::vector<int> deps = {s_glrt[k]};
                    const pl_batch_item& it = b->items[k];
                    for (int d = 0; d < it.N; ++d) {
                        const void* plane = it.planes ? (const void*)it.planes[d] : nullptr;
                        if (!plane) continue;
                        for (int j = 0; j < n; ++j)
                            if (j != k && b->items[j].kappa == plane) {
                                if (s_comp[j] < 0) return reject("an item reads the compressed SLC of a later level");
                                deps.push_back(s_comp[j]);
                            }
                    }
                    if ((int)deps.size() > kMegaMaxDeps) return reject("too many compressed SLCs from other items");
                    s_coh[k] = add(nt == 16 ? MS_COH16 : MS_COH32, (int)co.size() - 1, blocks, 1, deps);
                } else if (stage == 3) {
                    const int cls = (A.link.N + 3) / 4;
                    if (mega_link_lds(cls) > lds) lds = mega_link_lds(cls);
                    li.push_back(A.link);
                    s_link[k] = add(MS_LINK + cls, (int)li.size() - 1, A.link_blocks, kMegaLinkPerUnit, {s_coh[k]});
                } else if (stage == 4 && A.has_comp) {
                    cp.push_back(A.comp);
                    s_comp[k] = add(MS_COMPRESS, (int)cp.size() - 1, A.comp_blocks, kMegaCompressPerUnit, {s_link[k]});
                }
            }
        }
    }
    if (lds + 256 > max_lds_bytes()) return reject("LDS of one workgroup exceeded");
    std::vector<int64_t> start(seg.size() + 1, 0);
    for (size_t i = 0; i < seg.size(); ++i) start[i + 1] = start[i] + seg[i].units;
    // one device block: counters first (zeroed once, they only grow), then the tables
    auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t o_cnt = off; off = up(off + 64 + seg.size() * 8);
    const size_t o_seg = off; off = up(off + seg.size() * sizeof(MegaSeg));
    const size_t o_start = off; off = up(off + start.size() * 8);
    const size_t o_st = off; off = up(off + st.size() * sizeof(StatsArgs) + 1);
    const size_t o_gl = off; off = up(off + gl.size() * sizeof(GlrtArgs) + 1);
    const size_t o_co = off; off = up(off + co.size() * sizeof(CohArgs) + 1);
    const size_t o_li = off; off = up(off + li.size() * sizeof(LinkArgs) + 1);
    const size_t o_cp = off; off = up(off + cp.size() * sizeof(CompressArgs) + 1);
    void* mem = nullptr;
    pl_status r = hip_ok(hipMalloc(&mem, off), "pl_batch_plan: single-launch tables");
    if (r != PL_OK) return r;
    b->mega_mem = mem;
    unsigned char* base = static_cast<unsigned char*>(mem);
    auto put = [&](size_t o, const void* src, size_t bytes) {
        return bytes ? hip_ok(hipMemcpy(base + o, src, bytes, hipMemcpyHostToDevice), "pl_batch_plan: table upload")
                     : PL_OK;
    };
    if ((r = hip_ok(hipMemset(base + o_cnt, 0, 64 + seg.size() * 8), "pl_batch_plan: counters")) != PL_OK) return r;
    if ((r = put(o_seg, seg.data(), seg.size() * sizeof(MegaSeg))) != PL_OK) return r;
    if ((r = put(o_start, start.data(), start.size() * 8)) != PL_OK) return r;
    if ((r = put(o_st, st.data(), st.size() * sizeof(StatsArgs))) != PL_OK) return r;
    if ((r = put(o_gl, gl.data(), gl.size() * sizeof(GlrtArgs))) != PL_OK) return r;
    if ((r = put(o_co, co.data(), co.size() * sizeof(CohArgs))) != PL_OK) return r;
    if ((r = put(o_li, li.data(), li.size() * sizeof(LinkArgs))) != PL_OK) return r;
    if ((r = put(o_cp, cp.data(), cp.size() * sizeof(CompressArgs))) != PL_OK) return r;
    MegaPlan& p = b->mega;
    p.seg = reinterpret_cast<const MegaSeg*>(base + o_seg);
    p.seg_start = reinterpret_cast<const int64_t*>(base + o_start);
    p.nseg = (int)seg.size();
    p.total = start.back();
    p.stats = reinterpret_cast<const StatsArgs*>(base + o_st);
    p.glrt = reinterpret_cast<const GlrtArgs*>(base + o_gl);
    p.coh = reinterpret_cast<const CohArgs*>(base + o_co);
    p.link = reinterpret_cast<const LinkArgs*>(base + o_li);
    p.comp = reinterpret_cast<const CompressArgs*>(base + o_cp);
    p.queue = reinterpret_cast<unsigned long long*>(base + o_cnt);
    p.run = reinterpret_cast<unsigned int*>(base + o_cnt + 8);
    p.finished = reinterpret_cast<unsigned int*>(base + o_cnt + 12);
    p.error = reinterpret_cast<unsigned int*>(base + o_cnt + 16);
    p.done = reinterpret_cast<unsigned long long*>(base + o_cnt + 64);
    p.spin_limit = 1u << 20;  // about a quarter of a second of sleeping per wait
    b->mega_nseg = (int)seg.size();
    b->mega_lds = lds;
    if ((r = allow_dynamic_lds(mega_fn(b->split), lds)) != PL_OK) return r;
    int per_cu = 0;
    if ((r = hip_ok(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mega_fn(b->split), mega_threads(), lds),
                    "pl_batch_plan: occupancy query")) != PL_OK)
        return r;
    if (per_cu < 1) return reject("the single-launch kernel does not fit on a compute unit");
    b->mega_grid = (int64_t)per_cu * b->cus;
    b->single_ok = true;
    return PL_OK;
}

void destroy(pl_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto& L : b->levels) {
        for (auto& g : L.stats) release(g);
        release(L.glrt);
        for (auto& g : L.coh) release(g);
        for (auto& g : L.link) release(g);
        release(L.comp);
    }
    for (void* p : b->allocations) (void)hipFree(p);
    if (b->mega_mem) (void)hipFree(b->mega_mem);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->own) (void)hipStreamDestroy(b->own);
    delete b;
}

}  // namespace

#define PL_CHECK(cond, status, ...) \
    do {                            \
        if (!(cond)) return fail(status, __VA_ARGS__); \
    } while (0)

extern "C" {

pl_status pl_batch_plan(const pl_batch_item* items, int32_t n_items, pl_window w, double alpha,
                        pl_precision prec, pl_link_method method, int32_t tune, pl_stream stream,
                        pl_batch** out) {
    PL_CHECK(items && out, PL_ERR_INVALID_ARG, "pl_batch_plan: NULL pointer");
    PL_CHECK(n_items >= 1 && n_items <= 4096, PL_ERR_UNSUPPORTED, "pl_batch_plan: %d items (1..4096)", n_items);
    PL_CHECK(alpha > 0 && alpha < 1, PL_ERR_INVALID_ARG, "pl_batch_plan: alpha must lie in (0, 1)");
    PL_CHECK(prec == PL_PREC_FP32 || prec == PL_PREC_SPLIT_BF16, PL_ERR_INVALID_ARG,
             "pl_batch_plan: unknown precision %d", (int)prec);
    PL_CHECK(method == PL_LINK_EMI || method == PL_LINK_EVD, PL_ERR_INVALID_ARG,
             "pl_batch_plan: unknown method %d", (int)method);
    for (int k = 0; k < n_items; ++k) {
        const pl_batch_item& it = items[k];
        Geometry g;
        PL_CHECK((it.stack || it.planes) && it.phasors, PL_ERR_INVALID_ARG,
                 "pl_batch_plan: item %d: NULL stack or phasors", k);
        PL_CHECK(it.N >= 1 && it.N <= kMaxN, PL_ERR_UNSUPPORTED, "pl_batch_plan: item %d: N=%d outside 1..%d", k,
                 it.N, kMaxN);
        PL_CHECK(it.first_real >= 0 && it.first_real < it.N, PL_ERR_INVALID_ARG,
                 "pl_batch_plan: item %d: first_real %d outside 0..%d", k, it.first_real, it.N - 1);
        PL_CHECK(it.ref_idx >= 0 && it.ref_idx < it.N, PL_ERR_INVALID_ARG,
                 "pl_batch_plan: item %d: ref_idx %d outside 0..%d", k, it.ref_idx, it.N - 1);
        PL_CHECK((it.mean == nullptr) == (it.var == nullptr), PL_ERR_INVALID_ARG,
                 "pl_batch_plan: item %d: mean and var must both be given or both be NULL", k);
        PL_CHECK(make_geometry(it.R, it.C, w, &g) && g.oR >= 1 && g.oC >= 1, PL_ERR_SHAPE,
                 "pl_batch_plan: item %d: bad image size or window", k);
        PL_CHECK(g.R <= 2147483647LL, PL_ERR_UNSUPPORTED, "pl_batch_plan: item %d: too many rows", k);
        if (it.planes)
            for (int d = 0; d < it.N; ++d)
                PL_CHECK(it.planes[d], PL_ERR_INVALID_ARG, "pl_batch_plan: item %d: NULL plane %d", k, d);
    }
    pl_batch* b = new pl_batch();
    b->split = prec == PL_PREC_SPLIT_BF16;
    pl_status st = PL_OK;
    auto bail = [&](pl_status s) {
        destroy(b);
        return s;
    };
    {
        int dev = 0;
        st = hip_ok(hipGetDevice(&dev), "pl_batch_plan: device");
        if (st == PL_OK) st = hip_ok(hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev),
                                     "pl_batch_plan: device attribute");
        if (st == PL_OK) st = hip_ok(hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking), "pl_batch_plan: stream");
        if (st == PL_OK) st = hip_ok(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming), "pl_batch_plan: event");
        if (st == PL_OK) st = hip_ok(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming), "pl_batch_plan: event");
        if (st != PL_OK) return bail(st);
    }
    b->items.assign(items, items + n_items);
    b->iargs.assign(n_items, ItemArgs{});
    for (int k = 0; k < n_items; ++k) b->level_ids.push_back(items[k].level);
    std::sort(b->level_ids.begin(), b->level_ids.end());
    b->level_ids.erase(std::unique(b->level_ids.begin(), b->level_ids.end()), b->level_ids.end());
    b->levels.resize(b->level_ids.size());
    for (int k = 0; k < n_items; ++k) {
        const pl_batch_item& it = items[k];
        Level& L = b->levels[std::lower_bound(b->level_ids.begin(), b->level_ids.end(), it.level) - b->level_ids.begin()];
        Geometry g;
        make_geometry(it.R, it.C, w, &g);
        const int64_t P = g.oR * g.oC, px = g.R * g.C;
        auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
        const size_t o_mask = 0, o_count = up(o_mask + (size_t)P * g.nw * 4), o_coh = up(o_count + (size_t)P * 2);
        const size_t o_mean = up(o_coh + (size_t)P * it.N * it.N * 8);
        const size_t o_var = o_mean + (it.mean ? 0 : up((size_t)px * 8));
        const size_t bytes = o_var + (it.mean ? 0 : up((size_t)px * 8));
        void* mem = nullptr;
        st = hip_ok(hipMalloc(&mem, bytes), "pl_batch_plan: intermediates");
        if (st != PL_OK) return bail(st);
        b->allocations.push_back(mem);
        unsigned char* base = static_cast<unsigned char*>(mem);
        uint32_t* mask = reinterpret_cast<uint32_t*>(base + o_mask);
        uint16_t* count = reinterpret_cast<uint16_t*>(base + o_count);
        float2* coh = reinterpret_cast<float2*>(base + o_coh);
        const double* mean = it.mean;
        const double* var = it.var;
        PlaneTable t{};
        if (it.planes) {
            for (int d = 0; d < it.N; ++d) t.p[d] = reinterpret_cast<const float2*>(it.planes[d]);
        } else {
            t = contiguous_planes(it.stack, it.N, px);
        }
        if (!mean) {
            double* m = reinterpret_cast<double*>(base + o_mean);
            double* v = reinterpret_cast<double*>(base + o_var);
            StatsArgs a;
            int64_t blocks;
            const bool vec = stats_args(t, it.first_real, it.N - it.first_real, px, m, v, &a, &blocks);
            add_member(L.stats[vec ? 1 : 0], k, a, blocks);
            b->iargs[k].has_stats = true;
            b->iargs[k].stats_vec = vec;
            b->iargs[k].stats = a;
            b->iargs[k].stats_blocks = blocks;
            mean = m;
            var = v;
        }
        {
            GlrtArgs a;
            int64_t blocks;
            size_t lds;
            const double n_eff = it.n_eff > 0 ? it.n_eff : (double)(it.N - it.first_real);
            if (!glrt_args(mean, var, g, n_eff, alpha, mask, count, nullptr, &a, &blocks, &lds))
                return bail(fail(PL_ERR_UNSUPPORTED, "pl_batch_plan: window/stride too large for the GLRT tile"));
            add_member(L.glrt, k, a, blocks);
            b->iargs[k].glrt = a;
            b->iargs[k].glrt_blocks = blocks;
            b->iargs[k].glrt_lds = lds;
            L.glrt.threads = a.TX * a.TY;  // same window and stride for every item
            L.glrt.lds = lds;
        }
        {
            CohArgs a{};
            a.t = t;
            a.N = it.N;
            a.g = g;
            a.mask = mask;
            a.coh = coh;
            a.packed = 0;
            a.oy_lo = 0;
            a.oy_hi = g.oR;
            a.n_pairs = g.wy * (g.hx + 1);
            Group<CohArgs>& cg = L.coh[it.N <= 16 ? 0 : 1];
            cg.variant = it.N <= 16 ? 16 : 32;
            add_member(cg, k, a, 0);  // blocks set by configure_coherence
            b->iargs[k].coh = a;
        }
        {
            const LinkArgs a = link_args(coh, it.N, P, it.ref_idx, (int)method, reinterpret_cast<float2*>(it.phasors),
                                         nullptr, nullptr, it.flags, nullptr);
            Group<LinkArgs>& lg = L.link[(it.N + 3) / 4];
            lg.variant = (it.N + 3) / 4;
            add_member(lg, k, a, link_blocks(it.N, P));
            b->iargs[k].link = a;
            b->iargs[k].link_blocks = link_blocks(it.N, P);
        }
        if (it.kappa) {
            int64_t blocks;
            const CompressArgs a = compress_args(t, it.N, it.first_real, g, reinterpret_cast<const float2*>(it.phasors),
                                                 reinterpret_cast<float2*>(it.kappa), &blocks);
            add_member(L.comp, k, a, blocks);
            b->iargs[k].has_comp = true;
            b->iargs[k].comp = a;
            b->iargs[k].comp_blocks = blocks;
        }
    }
    for (auto& L : b->levels) {
        for (int v = 0; v < 2; ++v) {
            L.stats[v].threads = 256;
            if ((st = size_grid(b, L.stats[v], amp_stats_batch_fn(v == 1))) != PL_OK) return bail(st);
            if ((st = upload(L.stats[v])) != PL_OK) return bail(st);
        }
        if ((st = allow_dynamic_lds(glrt_batch_fn(), L.glrt.lds)) != PL_OK) return bail(st);
        if ((st = size_grid(b, L.glrt, glrt_batch_fn())) != PL_OK) return bail(st);
        if ((st = upload(L.glrt)) != PL_OK) return bail(st);
        for (int v = 0; v < 2; ++v) {
            Group<CohArgs>& g = L.coh[v];
            if (g.empty()) continue;
            g.threads = coherence_threads(g.variant);
            if ((st = configure_coherence(b, L, v, coherence_strip(g.variant), 0)) != PL_OK) return bail(st);
        }
        for (auto& g : L.link) {
            if (g.empty()) continue;
            g.threads = 256;
            if ((st = size_grid(b, g, phase_link_batch_fn(g.variant))) != PL_OK) return bail(st);
            if ((st = upload(g)) != PL_OK) return bail(st);
        }
        L.comp.threads = 256;
        if ((st = size_grid(b, L.comp, compress_batch_fn())) != PL_OK) return bail(st);
        if ((st = upload(L.comp)) != PL_OK) return bail(st);
    }
    if ((st = build_mega(b)) != PL_OK) return bail(st);
    b->single = b->single_ok;  // one launch per run unless it cannot be built
    if (tune) {
        // inputs written on the caller's stream are visible to the plan's stream
        st = hip_ok(hipEventRecord(b->ev_in, reinterpret_cast<hipStream_t>(stream)), "pl_batch_plan: event");
        if (st == PL_OK) st = hip_ok(hipStreamWaitEvent(b->own, b->ev_in, 0), "pl_batch_plan: event");
        if (st == PL_OK) st = autotune(b);
        // both forms on the live inputs, for the record (pl_batch_describe)
        if (st == PL_OK) {
            const bool keep = b->single;
            b->single = false;
            st = time_ms(b->own, [&] { return enqueue_all(b, b->own); }, 2, &b->graph_ms);
            if (st == PL_OK && b->single_ok) {
                b->single = true;
                st = time_ms(b->own, [&] { return enqueue_all(b, b->own); }, 2, &b->mega_ms);
            }
            b->single = keep;
        }
        if (st != PL_OK) return bail(st);
    }
    *out = b;
    return PL_OK;
}

pl_status pl_batch_run(pl_batch* b, pl_stream stream) {
    PL_CHECK(b, PL_ERR_INVALID_ARG, "pl_batch_run: NULL plan");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    pl_status st = hip_ok(hipEventRecord(b->ev_in, s), "pl_batch_run: event");
    if (st == PL_OK) st = hip_ok(hipStreamWaitEvent(b->own, b->ev_in, 0), "pl_batch_run: event");
    if (st != PL_OK) return st;
    if (!b->exec) {
        st = hip_ok(hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal), "pl_batch_run: graph capture");
        if (st != PL_OK) return st;
        const pl_status launched = enqueue_all(b, b->own);
        hipGraph_t graph = nullptr;
        st = hip_ok(hipStreamEndCapture(b->own, &graph), "pl_batch_run: graph capture");
        if (launched != PL_OK || st != PL_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return launched != PL_OK ? launched : st;
        }
        b->graph = graph;
        st = hip_ok(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "pl_batch_run: graph instantiate");
        if (st != PL_OK) return st;
    }
    st = hip_ok(hipGraphLaunch(b->exec, b->own), "pl_batch_run: graph launch");
    if (st == PL_OK) st = hip_ok(hipEventRecord(b->ev_out, b->own), "pl_batch_run: event");
    if (st == PL_OK) st = hip_ok(hipStreamWaitEvent(s, b->ev_out, 0), "pl_batch_run: event");
    if (st == PL_OK) ++b->runs;
    return st;
}

pl_status pl_batch_destroy(pl_batch* b) {
    if (!b) return PL_OK;
    (void)hipStreamSynchronize(b->own);
    destroy(b);
    return PL_OK;
}

pl_status pl_batch_set_single_launch(pl_batch* b, int32_t on) {
    PL_CHECK(b, PL_ERR_INVALID_ARG, "pl_batch_set_single_launch: NULL plan");
    PL_CHECK(!on || b->single_ok, PL_ERR_UNSUPPORTED, "pl_batch_set_single_launch: %s", b->single_why.c_str());
    if ((on != 0) == b->single) return PL_OK;
    pl_status st = hip_ok(hipStreamSynchronize(b->own), "pl_batch_set_single_launch: stream");
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->single = on != 0;
    return st;
}

pl_status pl_batch_check(pl_batch* b, pl_stream stream) {
    PL_CHECK(b, PL_ERR_INVALID_ARG, "pl_batch_check: NULL plan");
    pl_status st = hip_ok(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)), "pl_batch_check: stream");
    if (st == PL_OK) st = hip_ok(hipStreamSynchronize(b->own), "pl_batch_check: stream");
    if (st != PL_OK || !b->single_ok) return st;
    unsigned int err = 0;
    st = hip_ok(hipMemcpy(&err, b->mega.error, sizeof err, hipMemcpyDeviceToHost), "pl_batch_check: error word");
    if (st == PL_OK && err) {
        (void)hipMemset(b->mega.error, 0, sizeof err);  // reported once
        return fail(PL_ERR_STATE, "pl_batch_check: a single-launch run waited past its bound");
    }
    return st;
}

pl_status pl_batch_set_wait_limit(pl_batch* b, uint32_t spins) {
    PL_CHECK(b, PL_ERR_INVALID_ARG, "pl_batch_set_wait_limit: NULL plan");
    PL_CHECK(b->single_ok, PL_ERR_UNSUPPORTED, "pl_batch_set_wait_limit: %s", b->single_why.c_str());
    pl_status st = hip_ok(hipStreamSynchronize(b->own), "pl_batch_set_wait_limit: stream");
    if (b->exec) (void)hipGraphExecDestroy(b->exec);  // the limit is a launch argument
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->mega.spin_limit = spins;
    return st;
}

pl_status pl_batch_describe(const pl_batch* b, char* buf, size_t len) {
    PL_CHECK(b && buf && len > 0, PL_ERR_INVALID_ARG, "pl_batch_describe: NULL pointer");
    std::string s;
    char line[256];
    snprintf(line, sizeof line, "items %zu, CUs %d, runs %d, graph %s\n", b->items.size(), b->cus, b->runs,
             b->exec ? "captured" : "not yet");
    s += line;
    int launches = 0;
    for (size_t l = 0; l < b->levels.size(); ++l) {
        const Level& L = b->levels[l];
        snprintf(line, sizeof line, "level %d:\n", b->level_ids[l]);
        s += line;
        for (int v = 0; v < 2; ++v)
            if (!L.stats[v].empty()) {
                ++launches;
                snprintf(line, sizeof line, "  stats%s: %zu items, %lld blocks, grid %lld\n", v ? " (16-byte)" : "",
                         L.stats[v].members.size(), (long long)L.stats[v].total(), (long long)L.stats[v].grid);
                s += line;
            }
        ++launches;
        snprintf(line, sizeof line, "  glrt: %zu items, %lld blocks, grid %lld\n", L.glrt.members.size(),
                 (long long)L.glrt.total(), (long long)L.glrt.grid);
        s += line;
        for (auto& g : L.coh)
            if (!g.empty()) {
                ++launches;
                snprintf(line, sizeof line,
                         "  coherence tile %d%s: %zu items, strip %d, rows %d, %lld blocks, grid %lld, lds %zu, tuned %.3f ms\n",
                         g.variant, b->split ? " split-bf16" : " fp32", g.members.size(), g.txo, g.args[0].rows_per_wg,
                         (long long)g.total(), (long long)g.grid, g.lds, g.best_ms);
                s += line;
            }
        for (auto& g : L.link)
            if (!g.empty()) {
                ++launches;
                snprintf(line, sizeof line, "  link N<=%d: %zu items, %lld blocks, grid %lld (x%d), tuned %.3f ms\n",
                         4 * g.variant, g.members.size(), (long long)g.total(), (long long)g.grid, g.mult, g.best_ms);
                s += line;
            }
        if (!L.comp.empty()) {
            ++launches;
            snprintf(line, sizeof line, "  compress: %zu items, %lld blocks, grid %lld\n", L.comp.members.size(),
                     (long long)L.comp.total(), (long long)L.comp.grid);
            s += line;
        }
    }
    snprintf(line, sizeof line,
             "single launch: %s (%d segments, %lld work units, grid %lld, lds %zu), tuned %.3f ms; graph of the stage launches: tuned %.3f ms\n",
             b->single_ok ? "available" : b->single_why.c_str(), b->mega_nseg, (long long)b->mega.total,
             (long long)b->mega_grid, b->mega_lds, b->mega_ms, b->graph_ms);
    s += line;
    snprintf(line, sizeof line, "mode %s\nlaunches per run %d\n", b->single ? "single launch" : "stage launches",
             b->single ? 1 : launches);
    s += line;
    if (s.size() + 1 > len) s.resize(len - 1);
    snprintf(buf, len, "%s", s.c_str());
    return PL_OK;
}

}  // extern "C"
