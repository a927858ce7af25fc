// kubo_host.cpp -- the C ABI of include/kubo.h: validation, planning, workspace
// layout and the launch sequence.  No device arithmetic happens here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <tuple>
#include <vector>

#include "../../include/kubo.h"
#include "kubo_internal.h"
#include "kubo_launch.h"

using namespace kubo;

namespace {

constexpr size_t kAlign = 256;
constexpr int kCUs = 256;   // compute units of the MI355X
constexpr int kUnitK = 8;   // k-points per backward work unit
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Size classes of the per-k kernels (forward and adjoint alike): one wavefront
// per k-point with the matrices padded to np (n <= 32), or one workgroup per
// k-point with the matrices in workspace scratch (n <= 64: register
// back-transformation at two waves per SIMD; n <= 128: the LDS-staged one), or
// (n <= 512, forward only) the large-n pipeline, many workgroups per k-point.
struct ClassInfo {
    int np;
    bool wave;
    bool big;
};
const ClassInfo kClasses[] = {{8, true, false},   {16, true, false},   {32, true, false},
                              {64, false, false}, {128, false, false}, {512, false, true}};
constexpr int kNumClasses = sizeof(kClasses) / sizeof(kClasses[0]);

int class_of(int n) {
    for (int c = 0; c < kNumClasses; ++c)
        if (n <= kClasses[c].np) return c;
    return -1;
}

struct ClassRange {
    int begin = 0, count = 0;
    int max_k = 0;  // most k-points of one item
};

struct Chunk {
    int pencil_begin = 0, pencil_count = 0;
    int pgroup_begin = 0, pgroup_count = 0;
    int grange_begin = 0, grange_count = 0;
    ClassRange cls[kNumClasses];
    long long cls_kpts[kNumClasses] = {0};
    size_t tbytes = 0, pbytes = 0, xbytes = 0;
};

struct GraphKey {
    const void* p[6];
    double d[2];
    void* stream;
    bool operator==(const GraphKey& o) const {
        return std::memcmp(p, o.p, sizeof(p)) == 0 && d[0] == o.d[0] && d[1] == o.d[1] &&
               stream == o.stream;
    }
};

struct CachedGraph {
    bool valid = false;
    GraphKey key{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// k-points per pass of the large-n pipeline (KUBO_BIG_BATCH, default kBigBatch)
int big_batch() {
    const char* e = std::getenv("KUBO_BIG_BATCH");
    long b = e ? std::atol(e) : kBigBatch;
    return (int)std::min<long>(std::max<long>(b, 1), 4096);
}

size_t chunk_cap_bytes() {
    const char* e = std::getenv("KUBO_CHUNK_MB");
    long mb = e ? std::atol(e) : 2048;
    if (mb < 1) mb = 1;
    return (size_t)mb << 20;
}

}  // namespace

struct kubo_plan_s {
    uint32_t flags = 0;
    int n_models = 0, nF = 0;
    long long total_k = 0;
    std::vector<ModelDev> models;
    std::vector<int> r0val, grp_start, grp_r, grp_R1, grp_R2, grp_rho, negr;
    int max_nR = 0;
    long long max_nn = 0;
    // forward (partial Bloch sums only) and backward (plus pencil-sum buffers)
    // chunkings of the same k-blocks
    struct ChunkSet {
        std::vector<PencilItem> pencils;
        std::vector<PencilGroup> pgroups;
        std::vector<BlockItem> blocks;
        std::vector<GaccRange> granges;
        std::vector<Chunk> chunks;
        size_t max_t = 0, max_p = 0, max_x = 0;
        size_t tab_pencils = 0, tab_pgroups = 0, tab_blocks = 0, tab_granges = 0;
    } fwd, bwd;
    int n_slots = 0;
    int n_orb_total = 0;    // orbitals summed over the models (length of a spin array)
    long long t_elems = 0;  // complex elements of t (all models)
    // workspace layout
    size_t off_queues = 0, off_tables = 0, off_tp = 0, off_tbuf = 0, off_pbuf = 0, off_xbuf = 0, off_partial = 0,
           total = 0;
    size_t off_scratch = 0;
    size_t off_big = 0, big_bytes = 0;  // the large-n pipeline's slices
    int big_batch = kBigBatch;          // k-points per pass of it
    long long slot_elems = 0;
    int wg_groups = 512;
    int n_queues = 0;  // per-k kernel launches (forward chunks, then backward), 8 counters each
    std::vector<unsigned char> blob;
    size_t tab_off[10] = {0};
    unsigned long long id = 0;           // unique per plan (never reused)
    std::set<const void*> used_ws;       // workspaces this plan has run on
    CachedGraph graph_fwd, graph_bwd, graph_tensor;
    int max_groups = 2048;
    int max_group = 1;  // most lattice vectors sharing one R_x value
    // KUBO_F_TIMING: event pairs around per-k kernel launches
    struct TimeRec {
        int which;
        long long kpts;
        hipEvent_t start, stop;
    };
    std::vector<TimeRec> trec;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tpool;
    bool capturing = false;
    bool no_events = false;  // no event records (the no-allocation forward)
};

namespace {

Tables device_tables(const kubo_plan_s* p, unsigned char* ws, bool backward) {
    unsigned char* b = ws + p->off_tables;
    const kubo_plan_s::ChunkSet& cs = backward ? p->bwd : p->fwd;
    Tables t;
    t.models = reinterpret_cast<const ModelDev*>(b + p->tab_off[0]);
    t.r0val = reinterpret_cast<const int*>(b + p->tab_off[1]);
    t.grp_start = reinterpret_cast<const int*>(b + p->tab_off[2]);
    t.grp_r = reinterpret_cast<const int*>(b + p->tab_off[3]);
    t.grp_R1 = reinterpret_cast<const int*>(b + p->tab_off[4]);
    t.grp_R2 = reinterpret_cast<const int*>(b + p->tab_off[5]);
    t.negr = reinterpret_cast<const int*>(b + p->tab_off[6]);
    t.grp_rho = reinterpret_cast<const int*>(b + p->tab_off[9]);
    t.pencils = reinterpret_cast<const PencilItem*>(b + cs.tab_pencils);
    t.pgroups = reinterpret_cast<const PencilGroup*>(b + cs.tab_pgroups);
    t.blocks = reinterpret_cast<const BlockItem*>(b + cs.tab_blocks);
    t.granges = reinterpret_cast<const GaccRange*>(b + cs.tab_granges);
    return t;
}

template <class T>
void append_blob(std::vector<unsigned char>& blob, size_t& off, const std::vector<T>& v) {
    off = align_up(blob.size());
    blob.resize(off + std::max<size_t>(v.size() * sizeof(T), 1));
    if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
}

kubo_status build_plan(kubo_plan_s* P, const kubo_model_desc* models, int n_models, int nF,
                       uint32_t flags, const kubo_tile* tiles, int n_tiles) {
    P->flags = flags;
    P->n_models = n_models;
    P->nF = nF;
    std::map<int, kubo_tile> tile_of;
    for (int i = 0; i < n_tiles; ++i) tile_of[tiles[i].n_orb] = tiles[i];
    const size_t cap = chunk_cap_bytes();

    long long t_off = 0;
    int orb_off = 0;
    int slot = 0;
    const bool tensor = (flags & KUBO_F_TENSOR) != 0;
    // pencil partial sets per pencil: T and Ty, and Tz for the Hall tensor
    const int nsets = tensor ? 3 : 2;
    const int ncomp = tensor ? 4 : 1;
    // per model: tables and its pencils / blocks (in model order)
    struct PB {
        PencilItem pi;
        std::vector<BlockItem> blocks;   // forward k-blocks (the tile's k_block)
        std::vector<BlockItem> bblocks;  // backward k-blocks: longer, so fewer pencil partials
        size_t tbytes, pbytes;
        size_t pmat;    // backward: one k-block's pencil partials (bytes)
        size_t xbytes;  // backward: the per-k adjoint matrices
        int cls;
    };
    std::vector<PB> all;
    for (int m = 0; m < n_models; ++m) {
        const kubo_model_desc& d = models[m];
        ModelDev md{};
        md.n = d.n_orb;
        md.nR = d.n_R;
        md.N0 = d.grid[0];
        md.N1 = d.grid[1];
        md.N2 = d.grid[2];
        md.t_off = t_off;
        md.Nk = (long long)d.grid[0] * d.grid[1] * d.grid[2];
        md.f_off = m * nF;
        md.orb_off = orb_off;
        orb_off += d.n_orb;
        // distinct R_x values, ascending, and R grouped by them
        std::vector<int> xs;
        for (int r = 0; r < d.n_R; ++r) xs.push_back(d.R[3 * r]);
        std::sort(xs.begin(), xs.end());
        xs.erase(std::unique(xs.begin(), xs.end()), xs.end());
        md.nR0 = (int)xs.size();
        md.r0_first = (int)P->r0val.size();
        for (int x : xs) P->r0val.push_back(x);
        md.gs_first = (int)P->grp_start.size();
        md.grp_first = (int)P->grp_r.size();
        int acc = 0;
        for (int xi = 0; xi < (int)xs.size(); ++xi) {
            const int acc0 = acc;
            P->grp_start.push_back(acc);
            // the group's lattice vectors ordered by (R_y, R_z): the pencil sums take
            // each run of equal R_y as one R_z sum
            std::vector<int> rs;
            for (int r = 0; r < d.n_R; ++r)
                if (d.R[3 * r] == xs[xi]) rs.push_back(r);
            std::stable_sort(rs.begin(), rs.end(), [&](int u, int v) {
                return std::make_pair(d.R[3 * u + 1], d.R[3 * u + 2]) <
                       std::make_pair(d.R[3 * v + 1], d.R[3 * v + 2]);
            });
            for (int r : rs) {
                P->grp_r.push_back(r);
                P->grp_R1.push_back(d.R[3 * r + 1]);
                P->grp_R2.push_back(d.R[3 * r + 2]);
                P->grp_rho.push_back(xi);
                ++acc;
            }
            P->max_group = std::max(P->max_group, acc - acc0);
        }
        P->max_nR = std::max(P->max_nR, d.n_R);
        P->max_nn = std::max(P->max_nn, (long long)d.n_orb * d.n_orb);
        P->grp_start.push_back(acc);
        md.neg_first = (int)P->negr.size();
        std::map<std::tuple<int, int, int>, int> idx;
        for (int r = 0; r < d.n_R; ++r) idx[{d.R[3 * r], d.R[3 * r + 1], d.R[3 * r + 2]}] = r;
        for (int r = 0; r < d.n_R; ++r)
            P->negr.push_back(idx[{-d.R[3 * r], -d.R[3 * r + 1], -d.R[3 * r + 2]}]);

        // slab -> pencils -> blocks
        const long long kb = d.k_begin;
        const long long kc = d.k_count < 0 ? md.Nk - kb : d.k_count;
        const long long ke = kb + kc;
        // default k-block: 32 points for the one-wavefront classes, 8 for the
        // workgroup classes (a k-point costs milliseconds there, so smaller items
        // keep the end of a launch short)
        int kblock = std::min(d.grid[0], d.n_orb > 32 ? 8 : 32);
        auto ti = tile_of.find(d.n_orb);
        if (ti != tile_of.end()) kblock = std::min(d.grid[0], ti->second.k_block);
        if (d.n_orb > 128) kblock = 1;  // the large-n pipeline: one k-point per item
        // the backward writes one set of pencil partials per k-block and sums them
        // afterwards, so it takes blocks of about 32 points, balanced over the pencil
        const int nbb = (d.grid[0] + 31) / 32;
        const int kblock_b = std::max(kblock, (d.grid[0] + nbb - 1) / nbb);
        int cls = class_of(d.n_orb);
        if (ti != tile_of.end() && ti->second.threads == 256) {
            // the workgroup kernel forced: its smallest class that holds n
            for (int c2 = 0; c2 < kNumClasses; ++c2)
                if (!kClasses[c2].wave && d.n_orb <= kClasses[c2].np) {
                    cls = c2;
                    break;
                }
        }
        md.slot_first = slot;
        const long long nn = (long long)d.n_orb * d.n_orb;
        const size_t mat_bytes = (size_t)2 * md.nR0 * nn * 16;  // per backward k-block
        const size_t tset_bytes = (size_t)nsets * md.nR0 * nn * 16;  // per pencil
        if (kc > 0) {
            for (long long pc = kb / d.grid[0]; pc <= (ke - 1) / d.grid[0]; ++pc) {
                PB pb;
                pb.pi.model = m;
                pb.pi.i1 = (int)(pc % d.grid[1]);
                pb.pi.i2 = (int)(pc / d.grid[1]);
                pb.pi.pad = 0;
                pb.pi.tbuf_off = 0;
                pb.tbytes = tset_bytes;
                pb.pmat = mat_bytes;
                pb.cls = cls;
                long long a0 = std::max(kb - pc * d.grid[0], 0LL);
                long long a1 = std::min(ke - pc * d.grid[0], (long long)d.grid[0]);
                for (long long a = a0; a < a1; a += kblock) {
                    BlockItem bi{};
                    bi.model = m;
                    bi.i0 = (int)a;
                    bi.count = (int)std::min<long long>(kblock, a1 - a);
                    bi.slot = slot++;
                    bi.i1 = pb.pi.i1;
                    bi.i2 = pb.pi.i2;
                    pb.blocks.push_back(bi);
                }
                for (long long a = a0; a < a1; a += kblock_b) {
                    BlockItem bi{};
                    bi.model = m;
                    bi.i0 = (int)a;
                    bi.count = (int)std::min<long long>(kblock_b, a1 - a);
                    bi.slot = -1;  // no forward partial sums
                    bi.i1 = pb.pi.i1;
                    bi.i2 = pb.pi.i2;
                    pb.bblocks.push_back(bi);
                }
                pb.pbytes = mat_bytes * pb.bblocks.size();
                pb.xbytes = (size_t)3 * nn * 16 * (size_t)(a1 - a0);
                all.push_back(std::move(pb));
            }
        }
        md.slot_count = slot - md.slot_first;
        P->total_k += kc;
        P->models.push_back(md);
        t_off += (long long)d.n_R * nn;
    }
    P->t_elems = t_off;
    P->n_slots = slot;

    // chunks: consecutive pencils while the T region stays under the cap (and, backward,
    // the per-block pencil partials plus the per-k adjoint matrices under sixteen
    // times the cap: enough work per launch that the last round of the
    // persistent grid is a small fraction)
    auto chunkify = [&](bool with_p, kubo_plan_s::ChunkSet& cs) {
        Chunk cur;
        std::vector<std::vector<BlockItem>> cls_blocks(kNumClasses);
        auto flush = [&]() {
            if (cur.pencil_count == 0) return;
            // pencil groups: runs of one model and one k_z index, at most kPencilGroup long
            cur.pgroup_begin = (int)cs.pgroups.size();
            for (int p = cur.pencil_begin; p < cur.pencil_begin + cur.pencil_count;) {
                int q = p + 1;
                while (q < cur.pencil_begin + cur.pencil_count && q - p < kPencilGroup &&
                       cs.pencils[q].model == cs.pencils[p].model && cs.pencils[q].i2 == cs.pencils[p].i2)
                    ++q;
                cs.pgroups.push_back(PencilGroup{p, q - p});
                p = q;
            }
            cur.pgroup_count = (int)cs.pgroups.size() - cur.pgroup_begin;
            cur.grange_begin = (int)cs.granges.size();
            if (!with_p) {
                // forward: deal whole pencils round-robin into eight bins, one per XCD
                // share of the persistent grid, so every XCD sees the same mix of models
                // (not the large-n class: its batches take runs of one model in order)
                for (int c = 0; c < kNumClasses; ++c) {
                    if (kClasses[c].big) continue;
                    std::vector<BlockItem> bins[8];
                    int p = -1;
                    for (size_t i = 0; i < cls_blocks[c].size(); ++i) {
                        const BlockItem& b = cls_blocks[c][i];
                        if (i == 0 || b.tbuf_off != cls_blocks[c][i - 1].tbuf_off) ++p;
                        bins[p & 7].push_back(b);
                    }
                    cls_blocks[c].clear();
                    for (auto& bin : bins) cls_blocks[c].insert(cls_blocks[c].end(), bin.begin(), bin.end());
                }
            }
            for (int c = 0; c < kNumClasses; ++c) {
                cur.cls[c].begin = (int)cs.blocks.size();
                cur.cls[c].count = (int)cls_blocks[c].size();
                cur.cls_kpts[c] = 0;
                for (auto& b : cls_blocks[c]) {
                    const int bi = (int)cs.blocks.size();
                    cur.cls[c].max_k = std::max(cur.cls[c].max_k, b.count);
                    if (cs.granges.size() > (size_t)cur.grange_begin &&
                        cs.granges.back().model == b.model &&
                        cs.granges.back().begin + cs.granges.back().count == bi)
                        cs.granges.back().count++;
                    else
                        cs.granges.push_back(GaccRange{b.model, bi, 1, 0});
                    cs.blocks.push_back(b);
                    cur.cls_kpts[c] += b.count;
                }
                cls_blocks[c].clear();
            }
            cur.grange_count = (int)cs.granges.size() - cur.grange_begin;
            cs.max_t = std::max(cs.max_t, cur.tbytes);
            cs.max_p = std::max(cs.max_p, cur.pbytes);
            cs.max_x = std::max(cs.max_x, cur.xbytes);
            cs.chunks.push_back(cur);
            cur = Chunk();
            cur.pencil_begin = (int)cs.pencils.size();
        };
        cur.pencil_begin = 0;
        for (const auto& pb0 : all) {
            PB pb = pb0;
            if (cur.pencil_count > 0 &&
                (cur.tbytes + pb.tbytes > cap ||
                 (with_p && cur.pbytes + cur.xbytes + pb.pbytes + pb.xbytes > 4 * cap)))
                flush();
            PencilItem pi = pb.pi;
            pi.tbuf_off = (long long)(cur.tbytes / 16);
            long long poff = (long long)(cur.pbytes / 16);
            long long xoff = (long long)(cur.xbytes / 16);
            const long long mat = (long long)(pb.pmat / 16);
            const long long nn = (long long)models[pi.model].n_orb * models[pi.model].n_orb;
            for (auto& b : (with_p ? pb.bblocks : pb.blocks)) {
                b.tbuf_off = pi.tbuf_off;
                b.pbuf_off = with_p ? poff : 0;
                b.xbuf_off = -1;
                if (with_p) {
                    poff += mat;
                    b.xbuf_off = xoff;
                    b.xfull = kClasses[pb.cls].wave ? 0 : 1;
                    xoff += 3 * nn * b.count;
                }
                cls_blocks[pb.cls].push_back(b);
            }
            cs.pencils.push_back(pi);
            cur.pencil_count++;
            cur.tbytes += pb.tbytes;
            cur.pbytes += pb.pbytes;
            if (with_p) cur.xbytes += pb.xbytes;
        }
        flush();
    };
    chunkify(false, P->fwd);
    if (!(flags & KUBO_F_FORWARD_ONLY)) chunkify(true, P->bwd);

    // index tables, uploaded into the workspace on first use
    append_blob(P->blob, P->tab_off[0], P->models);
    append_blob(P->blob, P->tab_off[1], P->r0val);
    append_blob(P->blob, P->tab_off[2], P->grp_start);
    append_blob(P->blob, P->tab_off[3], P->grp_r);
    append_blob(P->blob, P->tab_off[4], P->grp_R1);
    append_blob(P->blob, P->tab_off[5], P->grp_R2);
    append_blob(P->blob, P->tab_off[6], P->negr);
    append_blob(P->blob, P->tab_off[9], P->grp_rho);
    for (kubo_plan_s::ChunkSet* cs : {&P->fwd, &P->bwd}) {
        append_blob(P->blob, cs->tab_pencils, cs->pencils);
        append_blob(P->blob, cs->tab_pgroups, cs->pgroups);
        append_blob(P->blob, cs->tab_blocks, cs->blocks);
        append_blob(P->blob, cs->tab_granges, cs->granges);
    }
    const size_t max_t = std::max(P->fwd.max_t, P->bwd.max_t);
    const size_t max_p = P->bwd.max_p;

    size_t off = kAlign;  // status word
    P->n_queues = (int)(P->fwd.chunks.size() + P->bwd.chunks.size()) * kNumClasses;
    P->off_queues = off;
    off = align_up(off + (size_t)P->n_queues * 8 * sizeof(unsigned));
    P->off_tables = off;
    off = align_up(off + P->blob.size());
    P->off_tp = off;
    off = align_up(off + (size_t)P->t_elems * 16);
    P->off_tbuf = off;
    off = align_up(off + max_t);
    P->off_pbuf = off;
    if (!(P->flags & KUBO_F_FORWARD_ONLY)) off = align_up(off + max_p);
    P->off_xbuf = off;
    if (!(P->flags & KUBO_F_FORWARD_ONLY)) off = align_up(off + P->bwd.max_x);
    P->off_partial = off;
    off = align_up(off + (size_t)P->n_slots * nF * ncomp * 8);
    P->n_orb_total = orb_off;
    {
        int nmax = 1;
        for (const auto& md : P->models)
            if (md.n <= 128) nmax = std::max(nmax, md.n);
        P->slot_elems = wg_slot_elems(nmax);
        // most work units of one launch (a backward item splits into units of
        // at most kUnitK k-points)
        int most = 1;
        for (const Chunk& c : P->fwd.chunks)
            for (int k = 0; k < kNumClasses; ++k) most = std::max(most, c.cls[k].count);
        for (const Chunk& c : P->bwd.chunks)
            for (int k = 0; k < kNumClasses; ++k) {
                const int uk = std::max(1, std::min(c.cls[k].max_k, kUnitK));
                most = std::max(most, c.cls[k].count * ((c.cls[k].max_k + uk - 1) / uk));
            }
        P->wg_groups = std::min(P->wg_groups, most);
        if (P->wg_groups >= 8) P->wg_groups &= ~7;  // whole XCD rounds
        // only the workgroup classes use the per-workgroup scratch
        bool any_wg = false;
        for (const kubo_plan_s::ChunkSet* cs : {&P->fwd, &P->bwd})
            for (const Chunk& c : cs->chunks)
                for (int k = 0; k < kNumClasses; ++k)
                    if (!kClasses[k].wave && !kClasses[k].big && c.cls[k].count > 0) any_wg = true;
        if (!any_wg) P->slot_elems = 0;
    }
    P->off_scratch = off;
    off = align_up(off + (size_t)P->wg_groups * (size_t)P->slot_elems * 16);
    // the large-n pipeline's per-k slices: room for a batch of up to kBigBatch
    // k-points of the largest such model, within four times the chunk cap
    P->big_bytes = 0;
    P->big_batch = big_batch();
    for (const auto& md : P->models) {
        if (md.n <= 128) continue;
        long long most_k = 0;
        for (const Chunk& c : P->fwd.chunks) most_k = std::max(most_k, (long long)c.cls[kNumClasses - 1].count);
        const size_t slice = (size_t)big_layout(md.n).per_k * 16;
        const size_t want = slice * (size_t)std::min<long long>(most_k, big_batch());
        P->big_bytes = std::max(P->big_bytes, std::max(slice, std::min(want, 4 * cap)));
    }
    P->off_big = off;
    off = align_up(off + P->big_bytes);
    P->total = off;
    return KUBO_OK;
}

kubo_status validate(const kubo_model_desc* models, int n_models, int nF, uint32_t flags,
                     const kubo_tile* tiles, int n_tiles) {
    if (!models || n_models < 1) return KUBO_E_INVALID;
    if (nF < 1 || nF > kMaxFermi) return KUBO_E_INVALID;
    if (flags & ~(KUBO_F_GRAPH | KUBO_F_TIMING | KUBO_F_FORWARD_ONLY | KUBO_F_TENSOR |
                  KUBO_F_DEBUG_SWEEPCAP))
        return KUBO_E_INVALID;
    if (n_tiles < 0 || (n_tiles > 0 && !tiles)) return KUBO_E_INVALID;
    for (int i = 0; i < n_tiles; ++i) {
        const kubo_tile& t = tiles[i];
        if (t.n_orb < 1 || t.n_orb > 128 || t.k_block < 1 || t.reserved != 0)
            return KUBO_E_INVALID;
        if (t.threads != 0 && t.threads != 64 && t.threads != 256) return KUBO_E_INVALID;
        if (t.threads == 64 && t.n_orb > 32) return KUBO_E_INVALID;
    }
    bool unsupported = false;
    for (int m = 0; m < n_models; ++m) {
        const kubo_model_desc& d = models[m];
        if (d.n_orb < 1 || d.n_R < 1 || !d.R) return KUBO_E_INVALID;
        for (int a = 0; a < 3; ++a)
            if (d.grid[a] < 1 || d.grid[a] > (1 << 20)) return KUBO_E_INVALID;
        const long long Nk = (long long)d.grid[0] * d.grid[1] * d.grid[2];
        if (d.k_begin < 0 || d.k_begin >= Nk) return KUBO_E_INVALID;
        if (d.k_count < -1 || d.k_count == 0) return KUBO_E_INVALID;
        if (d.k_count > 0 && d.k_begin + d.k_count > Nk) return KUBO_E_INVALID;
        std::set<std::tuple<int, int, int>> seen;
        std::set<int> xs;
        for (int r = 0; r < d.n_R; ++r) {
            auto key = std::make_tuple(d.R[3 * r], d.R[3 * r + 1], d.R[3 * r + 2]);
            if (!seen.insert(key).second) return KUBO_E_INVALID;
            xs.insert(d.R[3 * r]);
            for (int a = 0; a < 3; ++a)
                if (d.R[3 * r + a] == INT32_MIN) return KUBO_E_INVALID;
        }
        for (int r = 0; r < d.n_R; ++r)
            if (!seen.count(std::make_tuple(-d.R[3 * r], -d.R[3 * r + 1], -d.R[3 * r + 2])))
                return KUBO_E_INVALID;
        if (d.n_orb > kMaxOrb) unsupported = true;
        else if (class_of(d.n_orb) < 0) unsupported = true;
        // n > 128 runs the large-n pipeline, which has the forward only
        if (d.n_orb > 128 && (!(flags & KUBO_F_FORWARD_ONLY) || (flags & KUBO_F_TENSOR)))
            unsupported = true;
        if (xs.size() > 16) unsupported = true;
    }
    return unsupported ? KUBO_E_UNSUPPORTED : KUBO_OK;
}

#define HIP_TRY(x)                                  \
    do {                                            \
        if ((x) != hipSuccess) return KUBO_E_HIP;   \
    } while (0)

// Which plan's index tables a workspace holds.  Plans can take turns on one
// workspace (and every no-allocation call on a device shares one), so the
// owner is looked up on every call and the tables are uploaded again whenever
// another plan wrote its own there in between.  Keys are device addresses,
// unique across devices; owners are plan ids, never reused.
std::mutex g_ws_mu;
std::map<const void*, unsigned long long> g_ws_owner;
unsigned long long g_next_plan_id = 1;

kubo_status ensure_tables(kubo_plan_s* P, void* ws, hipStream_t s) {
    std::lock_guard<std::mutex> lock(g_ws_mu);
    auto it = g_ws_owner.find(ws);
    if (it != g_ws_owner.end() && it->second == P->id) return KUBO_OK;
    HIP_TRY(hipMemcpyAsync(static_cast<unsigned char*>(ws) + P->off_tables, P->blob.data(),
                           P->blob.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    g_ws_owner[ws] = P->id;
    P->used_ws.insert(ws);
    return KUBO_OK;
}

void forget_plan(const kubo_plan_s* P) {
    std::lock_guard<std::mutex> lock(g_ws_mu);
    for (auto it = g_ws_owner.begin(); it != g_ws_owner.end();)
        it = (it->second == P->id) ? g_ws_owner.erase(it) : std::next(it);
}

// Event pair around one per-k launch (only outside graph capture).
struct TimedScope {
    kubo_plan_s* P;
    hipStream_t s;
    bool on = false;
    kubo_plan_s::TimeRec rec{};
    // record_now = false: the caller records start_event() and stop_event() itself
    // (around one launch inside a pipeline) and files them with finish_recorded()
    TimedScope(kubo_plan_s* P_, hipStream_t s_, int which, long long kpts, bool record_now = true)
        : P(P_), s(s_) {
        if (!(P->flags & KUBO_F_TIMING) || P->capturing || P->no_events) return;
        if (P->tpool.empty()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess) return;
            if (hipEventCreate(&b) != hipSuccess) {
                (void)hipEventDestroy(a);
                return;
            }
            P->tpool.push_back({a, b});
        }
        rec.which = which;
        rec.kpts = kpts;
        rec.start = P->tpool.back().first;
        rec.stop = P->tpool.back().second;
        P->tpool.pop_back();
        on = !record_now || hipEventRecord(rec.start, s) == hipSuccess;
        if (!on) P->tpool.push_back({rec.start, rec.stop});
    }
    hipEvent_t start_event() const { return on ? rec.start : nullptr; }
    hipEvent_t stop_event() const { return on ? rec.stop : nullptr; }
    void finish_recorded() {
        if (!on) return;
        P->trec.push_back(rec);
        on = false;
    }
    void finish() {
        if (!on) return;
        if (hipEventRecord(rec.stop, s) == hipSuccess)
            P->trec.push_back(rec);
        else
            P->tpool.push_back({rec.start, rec.stop});
        on = false;
    }
};

// Grid of a workgroup-class launch: no more workgroups than the GPU holds at once
// (one per CU for n <= 128, which takes all 160 KB of LDS; two for n <= 64), since
// the work queue balances the items over the resident ones.
int wg_grid_cap(const kubo_plan_s* P, int k) {
    const int resident = kClasses[k].np > 64 ? kCUs : 2 * kCUs;
    return std::min(P->wg_groups, resident);
}

kubo_status enqueue_forward(kubo_plan_s* P, const double* t, const double* ef, double eta,
                            double kT, double* sigma, unsigned char* ws, hipStream_t s,
                            bool tensor = false, const double* spin = nullptr) {
    const Tables tb = device_tables(P, ws, false);
    unsigned* status = reinterpret_cast<unsigned*>(ws);
    double* tp = reinterpret_cast<double*>(ws + P->off_tp);
    double* tbuf = reinterpret_cast<double*>(ws + P->off_tbuf);
    double* partial = reinterpret_cast<double*>(ws + P->off_partial);
    double* scratch = reinterpret_cast<double*>(ws + P->off_scratch);
    const int max_iter = (P->flags & KUBO_F_DEBUG_SWEEPCAP) ? 1 : kMaxSweeps;
    unsigned* queues = reinterpret_cast<unsigned*>(ws + P->off_queues);
    HIP_TRY(launch_clear(status, queues, 8 * P->n_queues, s));
    HIP_TRY(launch_hermproj(tb, P->n_models, P->t_elems, t, tp, s));
    for (size_t ci = 0; ci < P->fwd.chunks.size(); ++ci) {
        const Chunk& c = P->fwd.chunks[ci];
        HIP_TRY(launch_pencil(tb, c.pgroup_begin, c.pgroup_count, P->max_nn, tp, tbuf, tensor, s));
        for (int k = 0; k < kNumClasses; ++k) {
            if (c.cls[k].count == 0) continue;
            TimedScope ts(P, s, tensor ? 2 : 0, c.cls_kpts[k]);
            if (kClasses[k].big) {
                // runs of items of one model, at most a batch's worth at a time
                const BlockItem* items = P->fwd.blocks.data();
                for (int i = c.cls[k].begin; i < c.cls[k].begin + c.cls[k].count;) {
                    const int m = items[i].model;
                    const int n = P->models[m].n;
                    const long long per_k = big_layout(n).per_k;
                    const int batch = (int)std::max<long long>(
                        1, std::min<long long>(P->big_batch, (long long)(P->big_bytes / 16) / per_k));
                    int j = i + 1;
                    while (j < c.cls[k].begin + c.cls[k].count && j - i < batch && items[j].model == m) ++j;
                    BigLaunch L{};
                    L.tb = tb;
                    L.tbuf = tbuf;
                    L.e_fermi = ef;
                    L.partial = partial;
                    L.status = status;
                    L.scratch = reinterpret_cast<double*>(ws + P->off_big);
                    L.per_k = per_k;
                    L.eta = eta;
                    L.kT = kT;
                    L.nF = P->nF;
                    L.n = n;
                    L.item_begin = i;
                    L.count = j - i;
                    TimedScope tr(P, s, 4, j - i, false);  // the reduction kernel alone
                    HIP_TRY(launch_big_forward(L, s, tr.start_event(), tr.stop_event()));
                    tr.finish_recorded();
                    i = j;
                }
            } else if (kClasses[k].wave) {
                FwdLaunch L;
                L.tb = tb;
                L.tbuf = tbuf;
                L.e_fermi = ef;
                L.partial = partial;
                L.status = status;
                L.eta = eta;
                L.kT = kT;
                L.nF = P->nF;
                L.max_sweeps = max_iter;
                L.item_begin = c.cls[k].begin;
                L.item_count = c.cls[k].count;
                L.np = kClasses[k].np;
                L.max_groups = P->max_groups;
                L.tensor = tensor ? 1 : 0;
                L.spin = spin;
                L.queue = queues + 8 * (ci * kNumClasses + k);
                HIP_TRY(launch_forward_wave(L, s));
            } else {
                WgLaunch L{};
                L.tb = tb;
                L.tbuf = tbuf;
                L.pbuf = nullptr;
                L.e_fermi = ef;
                L.sbar = nullptr;
                L.partial = partial;
                L.status = status;
                L.scratch = scratch;
                L.slot_elems = P->slot_elems;
                L.eta = eta;
                L.kT = kT;
                L.nF = P->nF;
                L.max_iter = max_iter;
                L.item_begin = c.cls[k].begin;
                L.item_count = c.cls[k].count;
                L.max_groups = wg_grid_cap(P, k);
                L.tensor = tensor ? 1 : 0;
                L.spin = spin;
                L.queue = queues + 8 * (ci * kNumClasses + k);
                L.unit_k = c.cls[k].max_k;
                L.unit_parts = 1;
                HIP_TRY(launch_forward_wg(L, kClasses[k].np, s));
            }
            ts.finish();
        }
    }
    HIP_TRY(launch_reduce(tb, P->n_models, P->nF, tensor ? 4 : 1, partial, sigma, status, s));
    return KUBO_OK;
}

// The Green's-function form: step 1 as in the forward, then k_gf per size class.
kubo_status enqueue_gf(kubo_plan_s* P, const double* t, const double* ef, double gamma,
                       const double* omega, const double* weight, int n_omega, double* sigma,
                       unsigned char* ws, hipStream_t s) {
    const Tables tb = device_tables(P, ws, false);
    unsigned* status = reinterpret_cast<unsigned*>(ws);
    double* tp = reinterpret_cast<double*>(ws + P->off_tp);
    double* tbuf = reinterpret_cast<double*>(ws + P->off_tbuf);
    double* partial = reinterpret_cast<double*>(ws + P->off_partial);
    unsigned* queues = reinterpret_cast<unsigned*>(ws + P->off_queues);
    HIP_TRY(launch_clear(status, queues, 8 * P->n_queues, s));
    HIP_TRY(launch_hermproj(tb, P->n_models, P->t_elems, t, tp, s));
    for (size_t ci = 0; ci < P->fwd.chunks.size(); ++ci) {
        const Chunk& c = P->fwd.chunks[ci];
        HIP_TRY(launch_pencil(tb, c.pgroup_begin, c.pgroup_count, P->max_nn, tp, tbuf, false, s));
        for (int k = 0; k < kNumClasses; ++k) {
            if (c.cls[k].count == 0) continue;
            TimedScope ts(P, s, 3, c.cls_kpts[k]);
            GfLaunch L{};
            L.tb = tb;
            L.tbuf = tbuf;
            L.e_fermi = ef;
            L.omega = omega;
            L.weight = weight;
            L.partial = partial;
            L.status = status;
            L.queue = queues + 8 * (ci * kNumClasses + k);
            L.gamma = gamma;
            L.nF = P->nF;
            L.n_omega = n_omega;
            L.item_begin = c.cls[k].begin;
            L.item_count = c.cls[k].count;
            L.max_groups = 3 * kCUs;  // three workgroups per CU (51 KB of LDS each)
            HIP_TRY(launch_gf(L, s));
            ts.finish();
        }
    }
    HIP_TRY(launch_reduce(tb, P->n_models, P->nF, 1, partial, sigma, status, s));
    return KUBO_OK;
}

kubo_status enqueue_backward(kubo_plan_s* P, const double* t, const double* ef, double eta,
                             double kT, const double* sbar, double* grad, unsigned char* ws,
                             hipStream_t s) {
    const Tables tb = device_tables(P, ws, true);
    unsigned* status = reinterpret_cast<unsigned*>(ws);
    double* tp = reinterpret_cast<double*>(ws + P->off_tp);
    double* tbuf = reinterpret_cast<double*>(ws + P->off_tbuf);
    double* pbuf = reinterpret_cast<double*>(ws + P->off_pbuf);
    double* xbuf = reinterpret_cast<double*>(ws + P->off_xbuf);
    double* scratch = reinterpret_cast<double*>(ws + P->off_scratch);
    const int max_iter = (P->flags & KUBO_F_DEBUG_SWEEPCAP) ? 1 : kMaxSweeps;
    unsigned* queues = reinterpret_cast<unsigned*>(ws + P->off_queues);
    HIP_TRY(launch_clear(status, queues, 8 * P->n_queues, s));
    HIP_TRY(launch_hermproj(tb, P->n_models, P->t_elems, t, tp, s));
    HIP_TRY(launch_zero(grad, 2 * P->t_elems, s));
    const size_t qbase = P->fwd.chunks.size();
    for (size_t ci = 0; ci < P->bwd.chunks.size(); ++ci) {
        const Chunk& c = P->bwd.chunks[ci];
        HIP_TRY(launch_pencil(tb, c.pgroup_begin, c.pgroup_count, P->max_nn, tp, tbuf, false, s));
        for (int k = 0; k < kNumClasses; ++k) {
            if (c.cls[k].count == 0) continue;
            WgLaunch L{};
            L.tb = tb;
            L.tbuf = tbuf;
            L.pbuf = pbuf;
            L.e_fermi = ef;
            L.sbar = sbar;
            L.partial = nullptr;
            L.status = status;
            L.scratch = scratch;
            L.xbuf = xbuf;
            L.slot_elems = P->slot_elems;
            L.eta = eta;
            L.kT = kT;
            L.nF = P->nF;
            L.max_iter = max_iter;
            L.item_begin = c.cls[k].begin;
            L.item_count = c.cls[k].count;
            L.max_groups = wg_grid_cap(P, k);
            L.queue = queues + 8 * ((qbase + ci) * kNumClasses + k);
            // work units of at most kUnitK k-points (a backward k-block is split),
            // so the end of a launch waits for a few k-points, not a whole block
            L.unit_k = std::min(c.cls[k].max_k, kUnitK);
            L.unit_parts = (c.cls[k].max_k + L.unit_k - 1) / L.unit_k;
            TimedScope ts(P, s, 1, c.cls_kpts[k]);
            if (kClasses[k].wave) {
                L.max_groups = P->max_groups;
                HIP_TRY(launch_adjoint_wave(L, kClasses[k].np, s));
            } else {
                HIP_TRY(launch_adjoint_wg(L, kClasses[k].np, s));
            }
            ts.finish();
            HIP_TRY(launch_pacc(tb, c.cls[k].begin, c.cls[k].count, P->max_nn, xbuf, pbuf, status, s));
        }
        HIP_TRY(launch_gacc(tb, tb.granges, c.grange_begin, c.grange_count, P->max_group, P->max_nn,
                            pbuf, grad, s));
    }
    HIP_TRY(launch_gsym(tb, P->n_models, P->t_elems, grad, s));
    return KUBO_OK;
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

// Capture the launch sequence into a hipGraph on first use (or when the key
// changes), then replay it.
template <class F>
kubo_status run_graph(kubo_plan_s* plan, CachedGraph& g, const GraphKey& key, hipStream_t s,
                      F&& enqueue) {
    if (!(g.valid && g.key == key)) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
        g = CachedGraph();
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        plan->capturing = true;
        kubo_status st = enqueue();
        plan->capturing = false;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(s, &graph);
        if (st != KUBO_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return KUBO_E_HIP;
        hipGraphExec_t exec = nullptr;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return KUBO_E_HIP;
        }
        g.graph = graph;
        g.exec = exec;
        g.key = key;
        g.valid = true;
    }
    HIP_TRY(hipGraphLaunch(g.exec, s));
    return KUBO_OK;
}

}  // namespace

namespace kubo {

kubo_status ahc_enqueue(kubo_plan_s* plan, const double* t, const double* e_fermi, double eta,
                        double kT, double* sigma, void* workspace, size_t workspace_bytes,
                        void* stream, bool allow_graph, bool tensor, const double* spin) {
    if (!plan || !t || !e_fermi || !sigma) return KUBO_E_INVALID;
    if (!finite_nonneg(eta) || !finite_nonneg(kT)) return KUBO_E_INVALID;
    if (tensor && !(plan->flags & KUBO_F_TENSOR)) return KUBO_E_INVALID;
    if (!workspace || workspace_bytes < plan->total) return KUBO_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    kubo_status st = ensure_tables(plan, workspace, s);
    if (st != KUBO_OK) return st;
    if (allow_graph && (plan->flags & KUBO_F_GRAPH) && s != nullptr) {
        GraphKey key{};
        key.p[0] = t;
        key.p[1] = e_fermi;
        key.p[2] = sigma;
        key.p[3] = workspace;
        key.p[5] = spin;
        key.d[0] = eta;
        key.d[1] = kT;
        key.stream = stream;
        return run_graph(plan, tensor ? plan->graph_tensor : plan->graph_fwd, key, s, [&]() {
            return enqueue_forward(plan, t, e_fermi, eta, kT, sigma, ws, s, tensor, spin);
        });
    }
    if (!allow_graph) {
        // no event records either: the caller may not be able to create them
        plan->no_events = true;
        st = enqueue_forward(plan, t, e_fermi, eta, kT, sigma, ws, s, tensor, spin);
        plan->no_events = false;
        return st;
    }
    return enqueue_forward(plan, t, e_fermi, eta, kT, sigma, ws, s, tensor, spin);
}

}  // namespace kubo

extern "C" {

kubo_status kubo_plan(kubo_plan_t* plan, const kubo_model_desc* models, int32_t n_models,
                      int32_t n_fermi, uint32_t flags, const kubo_tile* tiles, int32_t n_tiles,
                      size_t* workspace_bytes) {
    if (!plan || !workspace_bytes) return KUBO_E_INVALID;
    kubo_status st = validate(models, n_models, n_fermi, flags, tiles, n_tiles);
    if (st != KUBO_OK) return st;
    kubo_plan_s* P = new (std::nothrow) kubo_plan_s();
    if (!P) return KUBO_E_INVALID;
    st = build_plan(P, models, n_models, n_fermi, flags, tiles, n_tiles);
    if (st != KUBO_OK) {
        delete P;
        return st;
    }
    {
        std::lock_guard<std::mutex> lock(g_ws_mu);
        P->id = g_next_plan_id++;
    }
    *plan = P;
    *workspace_bytes = P->total;
    return KUBO_OK;
}

kubo_status kubo_ahc(kubo_plan_t plan, const double* t, const double* e_fermi, double eta,
                     double kT, double* sigma, void* workspace, size_t workspace_bytes,
                     void* stream) {
    return kubo::ahc_enqueue(plan, t, e_fermi, eta, kT, sigma, workspace, workspace_bytes, stream,
                             true);
}

kubo_status kubo_ahc_tensor(kubo_plan_t plan, const double* t, const double* e_fermi, double eta,
                            double kT, const double* spin, double* sigma, void* workspace,
                            size_t workspace_bytes, void* stream) {
    return kubo::ahc_enqueue(plan, t, e_fermi, eta, kT, sigma, workspace, workspace_bytes, stream,
                             true, true, spin);
}

kubo_status kubo_ahc_gf(kubo_plan_t plan, const double* t, const double* e_fermi, double gamma,
                        const double* omega, const double* weight, int32_t n_omega, double* sigma,
                        void* workspace, size_t workspace_bytes, void* stream) {
    if (!plan || !t || !e_fermi || !omega || !weight || !sigma) return KUBO_E_INVALID;
    if (!finite_nonneg(gamma) || n_omega < 1 || n_omega > KUBO_GF_MAX_NODES) return KUBO_E_INVALID;
    for (const auto& md : plan->models)
        if (md.n > 32) return KUBO_E_UNSUPPORTED;
    if (!workspace || workspace_bytes < plan->total) return KUBO_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    kubo_status st = ensure_tables(plan, workspace, s);
    if (st != KUBO_OK) return st;
    return enqueue_gf(plan, t, e_fermi, gamma, omega, weight, n_omega, sigma, ws, s);
}

kubo_status kubo_ahc_backward(kubo_plan_t plan, const double* t, const double* e_fermi,
                              double eta, double kT, const double* sigma_bar, double* grad_t,
                              void* workspace, size_t workspace_bytes, void* stream) {
    if (!plan || !t || !e_fermi || !sigma_bar || !grad_t) return KUBO_E_INVALID;
    if (plan->flags & KUBO_F_FORWARD_ONLY) return KUBO_E_INVALID;
    if (!finite_nonneg(eta) || !finite_nonneg(kT) || !(eta > 0.0)) return KUBO_E_INVALID;
    if (!workspace || workspace_bytes < plan->total) return KUBO_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char* ws = static_cast<unsigned char*>(workspace);
    kubo_status st = ensure_tables(plan, workspace, s);
    if (st != KUBO_OK) return st;
    if ((plan->flags & KUBO_F_GRAPH) && s != nullptr) {
        GraphKey key{};
        key.p[0] = t;
        key.p[1] = e_fermi;
        key.p[2] = sigma_bar;
        key.p[3] = workspace;
        key.p[4] = grad_t;
        key.d[0] = eta;
        key.d[1] = kT;
        key.stream = stream;
        return run_graph(plan, plan->graph_bwd, key, s, [&]() {
            return enqueue_backward(plan, t, e_fermi, eta, kT, sigma_bar, grad_t, ws, s);
        });
    }
    return enqueue_backward(plan, t, e_fermi, eta, kT, sigma_bar, grad_t, ws, s);
}

kubo_status kubo_plan_device_status(kubo_plan_t plan, const void* workspace, void* stream) {
    if (!plan || !workspace || !plan->used_ws.count(workspace)) return KUBO_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipStreamSynchronize(s) != hipSuccess) return KUBO_E_HIP;
    unsigned v = 0;
    if (hipMemcpy(&v, workspace, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return KUBO_E_HIP;
    if (v & kStatNoConv) return KUBO_E_NOCONV;
    if (v & kStatNonFinite) return KUBO_E_NONFINITE;
    return KUBO_OK;
}

kubo_status kubo_plan_kernel_time(kubo_plan_t plan, int32_t which, double* total_ms,
                                  int64_t* launches, int64_t* k_points, int32_t reset) {
    if (!plan || which < 0 || which > 4) return KUBO_E_INVALID;
    double ms = 0.0;
    long long nl = 0, kp = 0;
    for (const auto& r : plan->trec) {
        if (r.which != which) continue;
        if (hipEventSynchronize(r.stop) != hipSuccess) return KUBO_E_HIP;
        float e = 0.f;
        if (hipEventElapsedTime(&e, r.start, r.stop) != hipSuccess) return KUBO_E_HIP;
        ms += e;
        ++nl;
        kp += r.kpts;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = nl;
    if (k_points) *k_points = kp;
    if (reset) {
        std::vector<kubo_plan_s::TimeRec> keep;
        for (const auto& r : plan->trec) {
            if (r.which == which)
                plan->tpool.push_back({r.start, r.stop});
            else
                keep.push_back(r);
        }
        plan->trec.swap(keep);
    }
    return KUBO_OK;
}

void kubo_plan_destroy(kubo_plan_t plan) {
    if (!plan) return;
    for (const auto& r : plan->trec) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (const auto& e : plan->tpool) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (CachedGraph* g : {&plan->graph_fwd, &plan->graph_bwd, &plan->graph_tensor}) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
    }
    forget_plan(plan);
    delete plan;
}

const char* kubo_status_string(kubo_status status) {
    // a C caller may pass any int: read the value without loading an enum that C++
    // would consider out of range
    int32_t code = 0;
    std::memcpy(&code, &status, sizeof(code));
    switch (code) {
        case KUBO_OK:
            return "KUBO_OK";
        case KUBO_E_INVALID:
            return "KUBO_E_INVALID: argument out of range";
        case KUBO_E_UNSUPPORTED:
            return "KUBO_E_UNSUPPORTED: valid but not implemented";
        case KUBO_E_WORKSPACE:
            return "KUBO_E_WORKSPACE: workspace missing or too small";
        case KUBO_E_HIP:
            return "KUBO_E_HIP: HIP runtime call failed";
        case KUBO_E_NOCONV:
            return "KUBO_E_NOCONV: eigensolver hit its sweep cap";
        case KUBO_E_NONFINITE:
            return "KUBO_E_NONFINITE: non-finite value in the result";
    }
    return "unknown kubo_status";
}

kubo_status kubo_plan_info(kubo_plan_t plan, int64_t* total_k_points, int32_t* n_models) {
    if (!plan) return KUBO_E_INVALID;
    if (total_k_points) *total_k_points = plan->total_k;
    if (n_models) *n_models = plan->n_models;
    return KUBO_OK;
}

}  // extern "C"
