// Host side of the batch API declared in include/pdr.h (pdr_batch_*): many
// instances, each an ordinary context, swept together by the batched kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <string>
#include <utility>
#include <vector>

#include "pdr.h"
#include "pdr_context.h"
#include "pdr_internal.h"

using namespace pdr_host;
using pdr::Ctrl;
using pdr::Tiling;

// ------------------------------------------------------------------ batches
// A batch is a set of ordinary contexts (its members) on one stream and in one
// storage precision, plus batched kernels that run a pass of every member at
// once: one height launch whose blocks are apportioned to the members by work,
// one objective launch with a block per member (each member keeps its own stop
// test), and one arc launch per tiling bucket (members grouped by arc tiling,
// largest first). Per-member reads (flows, residual, z log) go through the
// member's own context.
struct pdr_batch {
    int32_t B = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t method = PDR_ESO;
    int32_t precision = PDR_FP64;
    int32_t graph_sweeps = 32;
    int32_t height_unroll = 4;
    int64_t height_budget = 0;  // height blocks of a batched pass, about
    std::vector<pdr_ctx *> members;
    pdr::InstView *d_views = nullptr;
    struct Bucket {
        Tiling tl{1, 1};
        std::vector<int32_t> members;  // largest m * Kp first
        int2 *d_amap = nullptr;        // (view index within the group, block) pairs
        int64_t nblocks = 0;
        int32_t max_K = 0;
        int64_t arcs = 0;
        double ms = 0.0;  // arc-kernel time of the last tuning run
        int32_t group = 0;
    };
    std::vector<Bucket> buckets;
    // Members are split into groups of about equal work; the views of a group
    // are contiguous in d_views, and each group's passes (height, objective,
    // its buckets' arc launches) run on a stream of their own, joined once per
    // batch of passes instead of once per pass.
    struct Group {
        int32_t off = 0, cnt = 0;  // views [off, off + cnt) of d_views
        int2 *d_hmap = nullptr;    // (view index within the group, block) pairs
        int64_t nhblocks = 0;
    };
    std::vector<Group> groups;
    std::vector<int32_t> vlocal;  // member -> view index within its group
    int32_t req_groups = 0;       // 0: automatic (kBranches, at most B)
    int32_t *d_count = nullptr;
    int32_t *h_count = nullptr;
    // group g's launches run on aux[g] (group 0 on the batch's stream),
    // forked from and joined back to the batch's stream with events
    static constexpr int kBranches = 4;
    hipStream_t aux[kBranches] = {};
    hipEvent_t fork = nullptr, join[kBranches] = {};
    hipStream_t cap_stream = nullptr;
    // One captured graph of graph_sweeps passes per group, each launched on
    // its group's stream: the runtime replays a graph's nodes on the stream it
    // is launched on, one after another, so branches inside one graph would
    // not overlap.
    hipGraphExec_t gexec[kBranches] = {};
    bool have_graphs = false;
    bool poisoned = false;
    std::string err;
};

namespace {

constexpr int64_t kBatchHeightBlocks = 32768;  // default height blocks of a batched pass
constexpr int32_t kBatchZLog = 4096;          // z log entries per member by default

pdr_status bfail(pdr_batch *b, pdr_status st, const std::string &msg)
{
    b->err = msg;
    return st;
}

pdr_status bdev_fail(pdr_batch *b, hipError_t e, const char *what)
{
    b->poisoned = true;
    b->err = std::string(what) + ": " + hipGetErrorString(e);
    return PDR_ERR_DEVICE;
}

#define PDR_BCHECK(b, expr)                                           \
    do {                                                              \
        hipError_t _e = (expr);                                       \
        if (_e != hipSuccess) return bdev_fail((b), _e, #expr);       \
    } while (0)

bool busable(pdr_batch *b, pdr_status *st)
{
    if (!b) {
        *st = PDR_ERR_INVALID;
        return false;
    }
    if (b->poisoned) {
        *st = PDR_ERR_DEVICE;
        return false;
    }
    hipError_t e = hipSetDevice(b->device);
    if (e != hipSuccess) {
        *st = bdev_fail(b, e, "hipSetDevice");
        return false;
    }
    return true;
}

// A member's failure belongs to the batch as well.
pdr_status member_fail(pdr_batch *b, int32_t i, pdr_status st)
{
    if (st == PDR_ERR_DEVICE) b->poisoned = true;
    b->err = "instance " + std::to_string(i) + ": " + b->members[i]->err;
    return st;
}

template <typename T>
hipError_t upload_vec(T **p, const std::vector<T> &v, hipStream_t st)
{
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (v.empty() ? 1 : v.size()));
    if (e == hipSuccess && !v.empty())
        e = hipMemcpyAsync(*p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

void drop_graph(pdr_batch *b)
{
    for (auto &ge : b->gexec) {
        if (ge) (void)hipGraphExecDestroy(ge);
        ge = nullptr;
    }
    b->have_graphs = false;
}

// Block map of one bucket with `lanes` lanes per arc: every member's arcs in
// blocks of arcs_per_block(lanes), members by their view index within the
// bucket's group (the order of the bucket's current map).
std::vector<int2> bucket_map(const pdr_batch *b, const pdr_batch::Bucket &bk, int lanes,
                             const std::vector<int32_t> &local)
{
    std::vector<int2> map;
    const int64_t apb = pdr::arcs_per_block(lanes);
    for (int32_t i : bk.members) {
        const int64_t nb = (b->members[i]->m + apb - 1) / apb;
        for (int64_t q = 0; q < nb; ++q) map.push_back(make_int2(local[i], (int)q));
    }
    return map;
}

// Rebuild the instance views, the groups, their height block maps and the
// tiling buckets from the members' current buffers and tilings.
pdr_status build_maps(pdr_batch *b)
{
    drop_graph(b);
    const int V = b->precision == PDR_FP64 ? 2 : 4;
    const int32_t B = b->B;
    std::vector<double> work(B);
    double W = 0.0;
    for (int32_t i = 0; i < B; ++i) {
        work[i] = (double)b->members[i]->n * (double)(b->members[i]->Kp / V);
        W += work[i];
    }
    // members largest first: the big ones start first and the small ones fill in
    std::vector<int32_t> order(B);
    for (int32_t i = 0; i < B; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return (double)b->members[x]->m * b->members[x]->Kp >
               (double)b->members[y]->m * b->members[y]->Kp;
    });
    // groups of about equal pass bytes (largest member to the lightest group)
    const int G = std::max(1, std::min<int>(b->req_groups > 0 ? b->req_groups
                                                                : pdr_batch::kBranches, B));
    std::vector<std::vector<int32_t>> gm(G);
    std::vector<double> load(G, 0.0);
    for (int32_t i : order) {
        const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        gm[g].push_back(i);
        load[g] += (double)b->members[i]->m * b->members[i]->Kp;
    }
    for (auto &grp : b->groups)
        if (grp.d_hmap) (void)hipFree(grp.d_hmap);
    b->groups.assign(G, pdr_batch::Group{});
    std::vector<pdr::InstView> views;
    views.reserve(B);
    std::vector<int32_t> local(B, 0);  // member -> view index within its group
    std::vector<int32_t> group_of(B, 0);
    for (int g = 0; g < G; ++g) {
        b->groups[g].off = (int32_t)views.size();
        b->groups[g].cnt = (int32_t)gm[g].size();
        for (int32_t i : gm[g]) {
            pdr_ctx *c = b->members[i];
            local[i] = (int32_t)views.size() - b->groups[g].off;
            group_of[i] = g;
            pdr::InstView v{};
            v.g = c->g;
            v.f = cur_f(c);
            v.h = cur_h(c);
            v.v = c->method == PDR_GDM ? cur_v(c) : nullptr;
            v.Fsum = c->Fsum;
            v.beta = c->beta;
            v.prm = agd_params(c);
            v.ctrl = c->ctrl;
            v.zpart = c->zpart;
            v.zlog = c->zlog;
            v.zmask = c->zlog_cap - 1;
            views.push_back(v);
        }
    }
    // about height_budget blocks in all, each member its share by work (at
    // least one block); every block grid-strides over its member's items
    const double budget = (double)b->height_budget;
    for (int g = 0; g < G; ++g) {
        std::vector<int2> hmap;
        for (int32_t i : gm[g]) {
            const int64_t need = std::max<int64_t>(1, (int64_t)std::ceil(work[i] / 256.0));
            const int64_t share =
                std::max<int64_t>(1, (int64_t)std::ceil(budget * work[i] / std::max(W, 1.0)));
            const int64_t nb = std::min<int64_t>({need, share, pdr::kHeightBlocksMax});
            views[b->groups[g].off + local[i]].nzpart = (int32_t)nb;
            for (int64_t q = 0; q < nb; ++q) hmap.push_back(make_int2(local[i], (int)q));
        }
        PDR_BCHECK(b, upload_vec(&b->groups[g].d_hmap, hmap, b->stream));
        b->groups[g].nhblocks = (int64_t)hmap.size();
    }
    PDR_BCHECK(b, upload_vec(&b->d_views, views, b->stream));
    b->vlocal = local;
    // tiling buckets, per group
    for (auto &bk : b->buckets)
        if (bk.d_amap) (void)hipFree(bk.d_amap);
    b->buckets.clear();
    for (int g = 0; g < G; ++g) {
        const size_t first = b->buckets.size();
        for (int32_t i : gm[g]) {
            const Tiling tl = b->members[i]->tiling;
            auto it = std::find_if(b->buckets.begin() + first, b->buckets.end(),
                                   [&](const pdr_batch::Bucket &x) {
                                       return x.tl.lanes == tl.lanes && x.tl.nv == tl.nv;
                                   });
            if (it == b->buckets.end()) {
                b->buckets.emplace_back();
                it = b->buckets.end() - 1;
                it->tl = tl;
                it->group = g;
            }
            it->members.push_back(i);
            it->max_K = std::max(it->max_K, b->members[i]->K);
            it->arcs += b->members[i]->m;
        }
    }
    for (auto &bk : b->buckets) {
        std::vector<int2> map;
        const int64_t apb = pdr::arcs_per_block(bk.tl.lanes);
        for (int32_t i : bk.members) {
            const int64_t nb = (b->members[i]->m + apb - 1) / apb;
            for (int64_t q = 0; q < nb; ++q) map.push_back(make_int2(local[i], (int)q));
        }
        PDR_BCHECK(b, upload_vec(&bk.d_amap, map, b->stream));
        bk.nblocks = (int64_t)map.size();
    }
    return PDR_OK;
}

// Views of a group, and of a bucket's group.
const pdr::InstView *group_views(const pdr_batch *b, int g) { return b->d_views + b->groups[g].off; }

// The height and objective launches of every group, one after another on st.
hipError_t enqueue_heights(pdr_batch *b, hipStream_t st)
{
    const bool fp64 = b->precision == PDR_FP64;
    for (size_t g = 0; g < b->groups.size(); ++g) {
        const auto &grp = b->groups[g];
        hipError_t e = pdr::launch_bheight(group_views(b, (int)g), grp.cnt, grp.d_hmap,
                                           grp.nhblocks, fp64, b->height_unroll, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The arc launches of one pass of every group, one after another on st.
hipError_t enqueue_batch_arcs(pdr_batch *b, hipStream_t st)
{
    const bool fp64 = b->precision == PDR_FP64;
    for (const auto &bk : b->buckets) {
        hipError_t e = pdr::launch_barc(b->method, group_views(b, bk.group), bk.d_amap,
                                        bk.nblocks, fp64, bk.tl, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// One batched pass of group g on sg: its height launch (objective and stop test
// included), then its buckets' arc launches.
hipError_t enqueue_group_pass(pdr_batch *b, int g, hipStream_t sg)
{
    const bool fp64 = b->precision == PDR_FP64;
    const auto &grp = b->groups[g];
    hipError_t e = pdr::launch_bheight(group_views(b, g), grp.cnt, grp.d_hmap, grp.nhblocks, fp64,
                                       b->height_unroll, sg);
    for (size_t k = 0; k < b->buckets.size() && e == hipSuccess; ++k) {
        const auto &bk = b->buckets[k];
        if (bk.group == g)
            e = pdr::launch_barc(b->method, group_views(b, g), bk.d_amap, bk.nblocks, fp64, bk.tl,
                                 sg);
    }
    return e;
}

// The group streams (group 0 on st, group g on aux[g]) wait for st...
hipError_t fork_groups(pdr_batch *b, hipStream_t st, hipStream_t *aux)
{
    const int G = (int)b->groups.size();
    hipError_t e = hipSuccess;
    if (G > 1) e = hipEventRecord(b->fork, st);
    for (int g = 1; g < G && e == hipSuccess; ++g) e = hipStreamWaitEvent(aux[g], b->fork, 0);
    return e;
}

// ... and st waits for them.
hipError_t join_groups(pdr_batch *b, hipStream_t st, hipStream_t *aux)
{
    hipError_t e = hipSuccess;
    for (int g = 1; g < (int)b->groups.size() && e == hipSuccess; ++g) {
        e = hipEventRecord(b->join[g], aux[g]);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, b->join[g], 0);
    }
    return e;
}

// `count` batched passes, each group's on a stream of its own, forked from st
// at the start and joined back at the end.
hipError_t enqueue_batch_passes(pdr_batch *b, int64_t count, hipStream_t st, hipStream_t *aux)
{
    const int G = (int)b->groups.size();
    hipError_t e = fork_groups(b, st, aux);
    for (int64_t q = 0; q < count && e == hipSuccess; ++q)
        for (int g = 0; g < G && e == hipSuccess; ++g)
            e = enqueue_group_pass(b, g, g == 0 ? st : aux[g]);
    if (e == hipSuccess) e = join_groups(b, st, aux);
    return e;
}

// Capture graph_sweeps passes of each group into a graph of its own.
pdr_status batch_graphs(pdr_batch *b)
{
    if (b->have_graphs) return PDR_OK;
    if (!b->cap_stream)
        PDR_BCHECK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    for (int g = 0; g < (int)b->groups.size(); ++g) {
        PDR_BCHECK(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int64_t q = 0; q < b->graph_sweeps && e == hipSuccess; ++q)
            e = enqueue_group_pass(b, g, b->cap_stream);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->cap_stream, &graph);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec[g], graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            drop_graph(b);
            PDR_BCHECK(b, e);
        }
    }
    b->have_graphs = true;
    return PDR_OK;
}

// graph_sweeps passes: every group's graph on its own stream.
hipError_t launch_batch_graphs(pdr_batch *b)
{
    hipError_t e = fork_groups(b, b->stream, b->aux);
    for (int g = 0; g < (int)b->groups.size() && e == hipSuccess; ++g)
        e = hipGraphLaunch(b->gexec[g], g == 0 ? b->stream : b->aux[g]);
    if (e == hipSuccess) e = join_groups(b, b->stream, b->aux);
    return e;
}

pdr_status count_stopped(pdr_batch *b, int32_t *n)
{
    PDR_BCHECK(b, pdr::launch_bcount_stopped(b->d_views, b->B, b->d_count, b->stream));
    PDR_BCHECK(b, hipMemcpyAsync(b->h_count, b->d_count, sizeof(int32_t), hipMemcpyDeviceToHost,
                                 b->stream));
    PDR_BCHECK(b, hipStreamSynchronize(b->stream));
    *n = *b->h_count;
    return PDR_OK;
}

void batch_free(pdr_batch *b)
{
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    for (auto &bk : b->buckets)
        if (bk.d_amap) (void)hipFree(bk.d_amap);
    b->buckets.clear();
    for (auto &grp : b->groups)
        if (grp.d_hmap) (void)hipFree(grp.d_hmap);
    b->groups.clear();
    for (pdr_ctx *c : b->members) {
        if (!c) continue;
        c->batch_member = false;
        pdr_destroy(c);
    }
    b->members.clear();
    if (b->d_views) (void)hipFree(b->d_views);
    if (b->d_count) (void)hipFree(b->d_count);
    if (b->h_count) (void)hipHostFree(b->h_count);
    b->d_views = nullptr;
    b->d_count = nullptr;
    b->h_count = nullptr;
    for (auto &x : b->aux)
        if (x) (void)hipStreamDestroy(x);
    for (auto &x : b->join)
        if (x) (void)hipEventDestroy(x);
    if (b->fork) (void)hipEventDestroy(b->fork);
    b->fork = nullptr;
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    b->cap_stream = nullptr;
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    b->stream = nullptr;
}

// Per-member snapshot of the run state an arc kernel changes (and the control
// record a height pass changes), for the tuner to put back.
struct Snapshot {
    std::vector<void *> bufs;
    ~Snapshot()
    {
        for (void *p : bufs) (void)hipFree(p);
    }
};

hipError_t snap_copy(Snapshot &sn, size_t slot, void *dst_or_src, size_t bytes, bool save,
                     hipStream_t st)
{
    if (save) {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, bytes ? bytes : 1);
        if (e != hipSuccess) return e;
        if (sn.bufs.size() <= slot) sn.bufs.resize(slot + 1, nullptr);
        sn.bufs[slot] = p;
        return hipMemcpyAsync(p, dst_or_src, bytes, hipMemcpyDeviceToDevice, st);
    }
    return hipMemcpyAsync(dst_or_src, sn.bufs[slot], bytes, hipMemcpyDeviceToDevice, st);
}

// Buffers saved per member: f, Fsum, beta, the control record, the z log (the
// tuner's whole passes write entries that, once the ring has wrapped, hold
// retained evaluations) and (GDM) v.
size_t slots_per_member(const pdr_batch *b) { return b->method == PDR_GDM ? 6 : 5; }

// Save (save = true) or restore the state of the listed members; a snapshot
// of every member in index order (the tuner's) keeps member i's buffers at
// slots [i * slots_per_member, ...).
hipError_t snapshot_members(pdr_batch *b, Snapshot &sn, const std::vector<int32_t> &mem, bool save)
{
    const size_t w = b->precision == PDR_FP64 ? 8 : 4;
    for (int32_t i : mem) {
        size_t slot = (size_t)i * slots_per_member(b);
        pdr_ctx *c = b->members[i];
        const size_t mK = (size_t)c->m * c->Kp;
        hipError_t e = snap_copy(sn, slot++, cur_f(c), mK * w, save, b->stream);
        if (e == hipSuccess) e = snap_copy(sn, slot++, c->Fsum, (size_t)c->m * 8, save, b->stream);
        if (e == hipSuccess) e = snap_copy(sn, slot++, c->beta, (size_t)c->m * 8, save, b->stream);
        if (e == hipSuccess) e = snap_copy(sn, slot++, c->ctrl, sizeof(Ctrl), save, b->stream);
        if (e == hipSuccess)
            e = snap_copy(sn, slot++, c->zlog, (size_t)c->zlog_cap * 8, save, b->stream);
        if (e == hipSuccess && c->method == PDR_GDM)
            e = snap_copy(sn, slot++, cur_v(c), mK * w, save, b->stream);
        if (e != hipSuccess) return e;
    }
    return hipStreamSynchronize(b->stream);
}

// Restore the arc-kernel state (f, Fsum, beta, v) of the listed members from a
// snapshot of every member; asynchronous on the batch stream.
hipError_t restore_members(pdr_batch *b, Snapshot &sn, const std::vector<int32_t> &mem)
{
    const size_t w = b->precision == PDR_FP64 ? 8 : 4;
    for (int32_t i : mem) {
        pdr_ctx *c = b->members[i];
        const size_t mK = (size_t)c->m * c->Kp, base = (size_t)i * slots_per_member(b);
        hipError_t e = snap_copy(sn, base, cur_f(c), mK * w, false, b->stream);
        if (e == hipSuccess) e = snap_copy(sn, base + 1, c->Fsum, (size_t)c->m * 8, false, b->stream);
        if (e == hipSuccess) e = snap_copy(sn, base + 2, c->beta, (size_t)c->m * 8, false, b->stream);
        if (e == hipSuccess && c->method == PDR_GDM)
            e = snap_copy(sn, base + 5, cur_v(c), mK * w, false, b->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

// *created receives the batch as soon as it exists, so that the exception
// barrier of pdr_batch_init can free it if the body is left part way.
static pdr_status pdr_batch_init_body(pdr_batch **out, int32_t B, const pdr_instance *insts,
                                      const pdr_options *opt_in, pdr_batch **created)
{
    if (!out) {
        g_init_error = "out is NULL";
        return PDR_ERR_INVALID;
    }
    *out = nullptr;
    if (B < 1 || !insts) {
        g_init_error = "a batch needs B >= 1 instances";
        return PDR_ERR_INVALID;
    }
    pdr_options opt;
    pdr_default_options(&opt);
    if (opt_in) opt = *opt_in;
    if (opt.height_blocks < 0 || opt.height_blocks > (1 << 20)) {
        g_init_error = "height_blocks of a batch must be 0 or 1..2^20";
        return PDR_ERR_INVALID;
    }
    if (opt.batch_groups < 0 || opt.batch_groups > pdr_batch::kBranches) {
        g_init_error = "batch_groups must be 0..4";
        return PDR_ERR_INVALID;
    }
    auto *b = new pdr_batch();
    *created = b;
    b->B = B;
    b->method = opt.method;
    b->precision = opt.precision;
    b->graph_sweeps = opt.graph_sweeps == 0 ? 32 : (opt.graph_sweeps < 0 ? 0 : opt.graph_sweeps);
    b->height_unroll = opt.height_unroll > 0 ? opt.height_unroll : kHeightUnrollAuto;
    b->height_budget = opt.height_blocks > 0 ? opt.height_blocks : kBatchHeightBlocks;
    b->req_groups = opt.batch_groups;
    auto init_fail_b = [&](pdr_status st, const std::string &msg) {
        g_init_error = msg;
        batch_free(b);
        delete b;
        return st;
    };
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) return init_fail_b(PDR_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (opt.stream) {
        b->stream = (hipStream_t)opt.stream;
    } else {
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return init_fail_b(PDR_ERR_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        b->own_stream = true;
    }
    pdr_options mo = opt;
    mo.stream = b->stream;
    mo.graph_sweeps = -1;
    mo.height_blocks = 0;  // the batch budget is not a member setting
    if (mo.z_log_capacity == 0) mo.z_log_capacity = kBatchZLog;
    b->members.assign(B, nullptr);
    for (int32_t i = 0; i < B; ++i) {
        const pdr_instance &in = insts[i];
        pdr_status st = pdr_init(&b->members[i], in.n, in.m, in.row_ptr, in.col, in.u, in.K, in.s,
                                 in.t, in.d, &mo);
        if (st != PDR_OK)
            return init_fail_b(st, "instance " + std::to_string(i) + ": " + g_init_error);
        b->members[i]->batch_member = true;
        set_cache_policy(b->members[i]);  // the batch's kernels stream
        if (b->members[i]->tiling.nv < 0)
            return init_fail_b(PDR_ERR_INVALID,
                               "instance " + std::to_string(i) +
                                   ": batches hold arc rows in registers (at most 8,192 vectors "
                                   "of 16 bytes: 16,384 commodities in FP64, 32,768 in FP32)");
    }
    e = hipMalloc((void **)&b->d_count, sizeof(int32_t));
    if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_count, sizeof(int32_t), hipHostMallocDefault);
    for (int r = 0; r < pdr_batch::kBranches && e == hipSuccess; ++r) {
        e = hipStreamCreateWithFlags(&b->aux[r], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[r], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    if (e != hipSuccess)
        return init_fail_b(e == hipErrorOutOfMemory ? PDR_ERR_OOM : PDR_ERR_DEVICE,
                           std::string("batch buffers: ") + hipGetErrorString(e));
    pdr_status st = build_maps(b);
    if (st != PDR_OK) return init_fail_b(st, b->err);
    *out = b;
    return PDR_OK;
}

static pdr_status pdr_batch_member_body(pdr_batch *b, int32_t index, pdr_ctx **ctx)
{
    pdr_status st;
    if (!busable(b, &st)) return st;
    if (!ctx || index < 0 || index >= b->B) return bfail(b, PDR_ERR_INVALID, "no such member");
    *ctx = b->members[index];
    return PDR_OK;
}

static pdr_status pdr_batch_sweep_body(pdr_batch *b, int64_t max_sweeps, double eps_obj, double z_target)
{
    pdr_status st;
    if (!busable(b, &st)) return st;
    if (max_sweeps < 0) return bfail(b, PDR_ERR_INVALID, "max_sweeps must be >= 0");
    if (std::isnan(eps_obj) || std::isnan(z_target))
        return bfail(b, PDR_ERR_INVALID, "eps_obj and z_target must not be NaN");
    PDR_BCHECK(b, pdr::launch_bbegin(b->d_views, b->B, eps_obj, z_target, b->stream));
    const bool poll = eps_obj > 0.0 || z_target > 0.0;
    const int64_t G = b->graph_sweeps;
    bool graphs = false;
    if (G > 0 && max_sweeps >= G) {
        st = batch_graphs(b);
        if (st != PDR_OK) return st;
        graphs = true;
    }
    int64_t s = 0, since = 0, every = 16;
    while (s < max_sweeps) {
        if (graphs && max_sweeps - s >= G) {
            PDR_BCHECK(b, launch_batch_graphs(b));
            s += G;
            since += G;
        } else {
            PDR_BCHECK(b, enqueue_batch_passes(b, 1, b->stream, b->aux));
            s += 1;
            since += 1;
        }
        if (poll && since >= every && s < max_sweeps) {
            since = 0;
            if (every < 1024) every *= 2;
            int32_t n = 0;
            st = count_stopped(b, &n);
            if (st != PDR_OK) return st;
            if (n == b->B) break;
        }
    }
    return PDR_OK;
}

static pdr_status pdr_batch_stopped_body(pdr_batch *b, int32_t *n_stopped)
{
    pdr_status st;
    if (!busable(b, &st)) return st;
    if (!n_stopped) return bfail(b, PDR_ERR_INVALID, "n_stopped is NULL");
    return count_stopped(b, n_stopped);
}

static pdr_status pdr_batch_buckets_body(pdr_batch *b, int32_t max_buckets, pdr_bucket_info *out,
                                         int32_t *n_buckets)
{
    pdr_status st;
    if (!busable(b, &st)) return st;
    if (!n_buckets || max_buckets < 0 || (max_buckets > 0 && !out))
        return bfail(b, PDR_ERR_INVALID, "bad bucket output");
    *n_buckets = (int32_t)b->buckets.size();
    for (int32_t q = 0; q < max_buckets && q < (int32_t)b->buckets.size(); ++q) {
        const auto &bk = b->buckets[q];
        out[q].lanes_per_arc = bk.tl.lanes;
        out[q].vec_per_lane = bk.tl.nv;
        out[q].instances = (int32_t)bk.members.size();
        out[q].max_K = bk.max_K;
        out[q].arcs = bk.arcs;
        out[q].ms = bk.ms;
    }
    return PDR_OK;
}

static pdr_status pdr_batch_tune_body(pdr_batch *b, int32_t reps, int64_t *height_blocks)
{
    pdr_status st;
    if (!busable(b, &st)) return st;
    if (reps < 1) return bfail(b, PDR_ERR_INVALID, "reps must be >= 1");
    const bool fp64 = b->precision == PDR_FP64;
    const int V = fp64 ? 2 : 4;
    std::vector<int32_t> all(b->B);
    for (int32_t i = 0; i < b->B; ++i) all[i] = i;
    // the starting configuration, kept if the tuned one is not faster
    std::vector<Tiling> start_tl(b->B);
    for (int32_t i = 0; i < b->B; ++i) start_tl[i] = b->members[i]->tiling;
    const int64_t start_budget = b->height_budget;
    Snapshot sn;
    PDR_BCHECK(b, snapshot_members(b, sn, all, true));
    // heights of the current flows, so the arc kernels see the real workload
    PDR_BCHECK(b, pdr::launch_bbegin(b->d_views, b->B, 0.0, 0.0, b->stream));
    PDR_BCHECK(b, enqueue_heights(b, b->stream));
    const int32_t start_groups = b->req_groups;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PDR_BCHECK(b, hipEventCreate(&e0));
    PDR_BCHECK(b, hipEventCreate(&e1));
    // a failure once timing launches have run leaves the saved state restored
    auto bail = [&](pdr_status why) -> pdr_status {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)snapshot_members(b, sn, all, false);
        return why;
    };
    std::vector<Tiling> best(b->buckets.size());
    hipError_t err = hipSuccess;
    for (size_t q = 0; q < b->buckets.size() && err == hipSuccess; ++q) {
        const auto &bk = b->buckets[q];
        int64_t maxvec = 1;
        for (int32_t i : bk.members) maxvec = std::max<int64_t>(maxvec, b->members[i]->Kp / V);
        const int64_t cap = 2 * (int64_t)pow2ceil(maxvec);
        double bms = std::numeric_limits<double>::infinity();
        Tiling bt = bk.tl;
        int2 *amap = nullptr;
        for (int L = 1; L <= kMaxLanes && err == hipSuccess; L *= 2)
            for (int nv = 1; nv <= kMaxNv && err == hipSuccess; ++nv) {
                if (!pdr::tiling_supported(L, nv) || (int64_t)L * nv < maxvec ||
                    (int64_t)L * nv > cap)
                    continue;
                const Tiling tl{L, nv};
                const std::vector<int2> map = bucket_map(b, bk, L, b->vlocal);
                err = upload_vec(&amap, map, b->stream);
                if (err != hipSuccess) break;
                // the same starting state for every candidate (only this
                // bucket's members change; the heights stay those computed above)
                err = restore_members(b, sn, bk.members);
                if (err == hipSuccess)
                    err = pdr::launch_barc(b->method, group_views(b, bk.group), amap,
                                           (int64_t)map.size(), fp64, tl, b->stream);
                if (err == hipSuccess) err = restore_members(b, sn, bk.members);
                if (err == hipSuccess) err = hipEventRecord(e0, b->stream);
                for (int r = 0; r < reps && err == hipSuccess; ++r)
                    err = pdr::launch_barc(b->method, group_views(b, bk.group), amap,
                                           (int64_t)map.size(), fp64, tl, b->stream);
                if (err == hipSuccess) err = hipEventRecord(e1, b->stream);
                if (err == hipSuccess) err = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
                if (err == hipSuccess && ms / reps < bms) {
                    bms = ms / reps;
                    bt = tl;
                }
            }
        if (amap) (void)hipFree(amap);
        best[q] = bt;
    }
    // each member's chosen tiling (the bucket list is rebuilt below)
    std::vector<Tiling> member_tl(b->B);
    for (size_t q = 0; q < b->buckets.size(); ++q)
        for (int32_t i : b->buckets[q].members) member_tl[i] = best[q];
    // the height launch: blocks in all (each member's share by work)
    int64_t best_budget = b->height_budget;
    double best_hms = std::numeric_limits<double>::infinity();
    for (int64_t cand = 8192; cand <= 65536 && err == hipSuccess; cand *= 2) {
        b->height_budget = cand;
        st = build_maps(b);
        if (st != PDR_OK) return bail(st);
        err = enqueue_heights(b, b->stream);
        if (err == hipSuccess) err = hipEventRecord(e0, b->stream);
        for (int r = 0; r < reps && err == hipSuccess; ++r) err = enqueue_heights(b, b->stream);
        if (err == hipSuccess) err = hipEventRecord(e1, b->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err == hipSuccess && ms / reps < best_hms) {
            best_hms = ms / reps;
            best_budget = cand;
        }
    }
    // The pieces were timed alone; a pass runs the buckets side by side after
    // the height launch. Time whole passes (from the saved state, stop tests
    // off) with the tuned and with the starting configuration and keep the
    // faster.
    auto apply = [&](const std::vector<Tiling> &tl, int64_t budget, int32_t groups) -> pdr_status {
        for (int32_t i = 0; i < b->B; ++i) b->members[i]->tiling = tl[i];
        b->height_budget = budget;
        b->req_groups = groups;
        return build_maps(b);
    };
    auto time_passes = [&](double *ms_out) -> hipError_t {
        hipError_t e = snapshot_members(b, sn, all, false);
        if (e == hipSuccess) e = pdr::launch_bbegin(b->d_views, b->B, 0.0, 0.0, b->stream);
        if (e == hipSuccess) e = enqueue_batch_passes(b, 1, b->stream, b->aux);
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        if (e == hipSuccess) e = enqueue_batch_passes(b, reps, b->stream, b->aux);
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        *ms_out = (double)ms / reps;
        return e;
    };
    // candidates: the tuned tilings and height blocks with the members in one
    // group and in kBranches groups, and the starting configuration
    struct Cand {
        const std::vector<Tiling> *tl;
        int64_t budget;
        int32_t groups;
        double ms;
    };
    std::vector<Cand> cands = {{&member_tl, best_budget, pdr_batch::kBranches, 0.0},
                               {&member_tl, best_budget, 1, 0.0},
                               {&start_tl, start_budget, start_groups, 0.0}};
    for (size_t q = 0; q < cands.size() && err == hipSuccess; ++q) {
        st = apply(*cands[q].tl, cands[q].budget, cands[q].groups);
        if (st != PDR_OK) return bail(st);
        err = time_passes(&cands[q].ms);
    }
    if (err == hipSuccess) {
        // the fastest stays; the starting configuration unless another beats it
        size_t pick = cands.size() - 1;
        for (size_t q = 0; q + 1 < cands.size(); ++q)
            if (cands[q].ms < cands[pick].ms) pick = q;
        st = apply(*cands[pick].tl, cands[pick].budget, cands[pick].groups);
        if (st != PDR_OK) return bail(st);
    }
    // each final bucket's arc launch on the saved state, for pdr_batch_buckets
    for (auto &bk : b->buckets) {
        if (err != hipSuccess) break;
        err = restore_members(b, sn, bk.members);
        if (err == hipSuccess) err = hipEventRecord(e0, b->stream);
        for (int r = 0; r < reps && err == hipSuccess; ++r)
            err = pdr::launch_barc(b->method, group_views(b, bk.group), bk.d_amap, bk.nblocks,
                                   fp64, bk.tl, b->stream);
        if (err == hipSuccess) err = hipEventRecord(e1, b->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        bk.ms = (double)ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err == hipSuccess) err = snapshot_members(b, sn, all, false);
    PDR_BCHECK(b, err);
    if (height_blocks) *height_blocks = b->height_budget;
    return PDR_OK;
}

static pdr_status pdr_batch_profile_sweeps_body(pdr_batch *b, int64_t sweeps, double *kernel_ms)
{
    pdr_status st;
    if (!busable(b, &st)) return st;
    if (sweeps < 0 || !kernel_ms) return bfail(b, PDR_ERR_INVALID, "bad arguments");
    hipEvent_t ev[3];
    for (auto &x : ev) PDR_BCHECK(b, hipEventCreate(&x));
    double tot[2] = {0.0, 0.0};
    hipError_t err = pdr::launch_bbegin(b->d_views, b->B, 0.0, 0.0, b->stream);
    for (int64_t s0 = 0; s0 < sweeps && err == hipSuccess; ++s0) {
        err = hipEventRecord(ev[0], b->stream);
        if (err == hipSuccess) err = enqueue_heights(b, b->stream);
        if (err == hipSuccess) err = hipEventRecord(ev[1], b->stream);
        if (err == hipSuccess) err = enqueue_batch_arcs(b, b->stream);
        if (err == hipSuccess) err = hipEventRecord(ev[2], b->stream);
        if (err == hipSuccess) err = hipEventSynchronize(ev[2]);
        for (int r = 0; r < 2 && err == hipSuccess; ++r) {
            float ms = 0.0f;
            err = hipEventElapsedTime(&ms, ev[r], ev[r + 1]);
            tot[r] += ms;
        }
    }
    for (auto &x : ev) (void)hipEventDestroy(x);
    PDR_BCHECK(b, err);
    kernel_ms[0] = tot[0];
    kernel_ms[1] = tot[1];
    return PDR_OK;
}

static pdr_status pdr_batch_set_precision_body(pdr_batch *b, int32_t precision)
{
    pdr_status st;
    if (!busable(b, &st)) return st;
    if (precision != PDR_FP64 && precision != PDR_FP32_BULK)
        return bfail(b, PDR_ERR_INVALID, "unknown precision");
    const int64_t maxvec = pdr::max_tiling_vectors();
    for (int32_t i = 0; i < b->B; ++i)  // batches hold rows in registers
        if (b->members[i]->Kp / (precision == PDR_FP64 ? 2 : 4) > maxvec)
            return bfail(b, PDR_ERR_INVALID,
                         "instance " + std::to_string(i) +
                             ": its row is longer than a batch holds in this precision");
    for (int32_t i = 0; i < b->B; ++i) {
        st = set_precision_impl(b->members[i], precision);
        if (st != PDR_OK) return member_fail(b, i, st);
    }
    b->precision = precision;
    return build_maps(b);
}

const char *pdr_batch_last_error(const pdr_batch *b)
{
    if (!b) return g_init_error.c_str();
    return b->err.c_str();
}

static void pdr_batch_destroy_body(pdr_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    batch_free(b);
    delete b;
}

}  // extern "C"

// ------------------------------------------------------------------ exported entry points
// Each runs its body behind the exception barrier (abi_guard).
extern "C" {

pdr_status pdr_batch_init(pdr_batch **out, int32_t B, const pdr_instance *insts,
                          const pdr_options *opt_in)
{
    pdr_batch *created = nullptr;
    bool returned = false;
    const pdr_status st = abi_guard(nullptr, nullptr, [&] {
        const pdr_status r = pdr_batch_init_body(out, B, insts, opt_in, &created);
        returned = true;
        return r;
    });
    if (!returned) {  // left part way by an exception: free what was built
        if (created) {
            try {
                batch_free(created);
            } catch (...) {
            }
            delete created;
        }
        if (out) *out = nullptr;
    }
    return st;
}

pdr_status pdr_batch_member(pdr_batch *b, int32_t index, pdr_ctx **ctx)
{
    return abi_guard(b ? &b->err : nullptr, nullptr,
                     [&] { return pdr_batch_member_body(b, index, ctx); });
}

pdr_status pdr_batch_sweep(pdr_batch *b, int64_t max_sweeps, double eps_obj, double z_target)
{
    return abi_guard(b ? &b->err : nullptr, b ? &b->poisoned : nullptr,
                     [&] { return pdr_batch_sweep_body(b, max_sweeps, eps_obj, z_target); });
}

pdr_status pdr_batch_stopped(pdr_batch *b, int32_t *n_stopped)
{
    return abi_guard(b ? &b->err : nullptr, nullptr,
                     [&] { return pdr_batch_stopped_body(b, n_stopped); });
}

pdr_status pdr_batch_buckets(pdr_batch *b, int32_t max_buckets, pdr_bucket_info *out,
                             int32_t *n_buckets)
{
    return abi_guard(b ? &b->err : nullptr, nullptr,
                     [&] { return pdr_batch_buckets_body(b, max_buckets, out, n_buckets); });
}

pdr_status pdr_batch_tune(pdr_batch *b, int32_t reps, int64_t *height_blocks)
{
    return abi_guard(b ? &b->err : nullptr, b ? &b->poisoned : nullptr,
                     [&] { return pdr_batch_tune_body(b, reps, height_blocks); });
}

pdr_status pdr_batch_profile_sweeps(pdr_batch *b, int64_t sweeps, double *kernel_ms)
{
    return abi_guard(b ? &b->err : nullptr, b ? &b->poisoned : nullptr,
                     [&] { return pdr_batch_profile_sweeps_body(b, sweeps, kernel_ms); });
}

pdr_status pdr_batch_set_precision(pdr_batch *b, int32_t precision)
{
    return abi_guard(b ? &b->err : nullptr, b ? &b->poisoned : nullptr,
                     [&] { return pdr_batch_set_precision_body(b, precision); });
}

void pdr_batch_destroy(pdr_batch *b)
{
    try {
        pdr_batch_destroy_body(b);
    } catch (...) {  // teardown cannot report; nothing may leave the ABI
    }
}

}  // extern "C"
