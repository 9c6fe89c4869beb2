// Batched application of many independent SIPG operators (sipg_batch_*).
//
// Operators are grouped by (degree, basis, precision, kernel geometry
// variant: per point, per cell, per cell with a diagonal metric); each
// group becomes one grid over the concatenated workgroup lists of its
// operators, so a batch of small operators fills the 256 compute units that
// each of them alone would leave mostly idle.  The per-operator kernel
// parameters and the workgroup -> operator table live in one device buffer
// made at creation; sipg_batch_apply only launches (one kernel per group).
// The groups are spread over the caller's stream and up to three more
// streams of the batch (default priority), forked from and joined back into
// the caller's stream with events, so that the grids of different groups run
// concurrently and the small ones fill the compute units the large ones leave
// idle at their ends.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "matvec.hpp"
#include "setup.hpp"
#include "sipg_common.hpp"

struct sipg_batch {
    int device = 0;
    int nops = 0;
    int64_t ndofs = 0, ncells = 0, nblocks = 0;
    std::vector<sipg::BatchGroup> groups;
    // per group: its operators and vectors (host copies), and the schedule
    // chosen by sipg_batch_tune (0: one grid, 1: one launch per operator)
    std::vector<std::vector<int>> members;
    std::vector<int> schedule;
    std::vector<const sipg_op*> ops;
    std::vector<const void*> x;
    std::vector<void*> y;
    void* mem = nullptr;
    sipg::DevAlloc alloc;           // provider of mem (the first operator's)
    // concurrent groups: stream of each group (0 = the caller's, j > 0 =
    // aux[j - 1]), and the fork / join events
    std::vector<int> lane;
    std::vector<hipStream_t> aux;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    size_t bytes = 0;
};

namespace sipg {

int launch_matvec_batched(const BatchGroup& g, hipStream_t st) {
    switch (g.n) {
        case 2: return launch_matvec_batched_n<2>(g, st);
        case 3: return launch_matvec_batched_n<3>(g, st);
        case 4: return launch_matvec_batched_n<4>(g, st);
        case 5: return launch_matvec_batched_n<5>(g, st);
        case 6: return launch_matvec_batched_n<6>(g, st);
        case 7: return launch_matvec_batched_n<7>(g, st);
        case 8: return launch_matvec_batched_n<8>(g, st);
        case 9: return launch_matvec_batched_n<9>(g, st);
    }
    set_error("unsupported degree");
    return SIPG_E_UNSUPPORTED;
}

namespace {

struct Range {
    const char* lo;
    const char* hi;
    int op;
    bool write;
};

// Any written range that meets another range (read or written) of a
// different role is a race inside one launch.
bool ranges_conflict(std::vector<Range> r, std::string& why) {
    std::sort(r.begin(), r.end(), [](const Range& a, const Range& b) { return a.lo < b.lo; });
    // sweep: keep the range with the largest end seen so far among writes and
    // among reads
    const Range* last_w = nullptr;
    const Range* last_any = nullptr;
    for (const Range& c : r) {
        if (last_w && c.lo < last_w->hi) {
            why = "the output of operator " + std::to_string(last_w->op) + " overlaps " +
                  (c.write ? "the output" : "the input") + " of operator " + std::to_string(c.op);
            return true;
        }
        if (c.write && last_any && c.lo < last_any->hi) {
            why = "the output of operator " + std::to_string(c.op) + " overlaps " +
                  (last_any->write ? "the output" : "the input") + " of operator " + std::to_string(last_any->op);
            return true;
        }
        if (c.write && (!last_w || c.hi > last_w->hi)) last_w = &c;
        if (!last_any || c.hi > last_any->hi) last_any = &c;
    }
    return false;
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace
}  // namespace sipg

using namespace sipg;

extern "C" {

int sipg_batch_create(int nops, const sipg_op* const* ops, const void* const* x, void* const* y,
                      sipg_batch** out) {
    if (!out) { set_error("sipg_batch_create: null output handle"); return SIPG_E_ARG; }
    *out = nullptr;
    if (nops <= 0 || !ops || !x || !y) { set_error("sipg_batch_create: empty batch or null array"); return SIPG_E_ARG; }
    std::vector<Range> ranges;
    ranges.reserve(2 * size_t(nops));
    int device = -1;
    for (int i = 0; i < nops; ++i) {
        if (!ops[i] || !x[i] || !y[i]) {
            set_error("sipg_batch_create: null operator or vector at entry " + std::to_string(i));
            return SIPG_E_ARG;
        }
        if (ops[i]->mesh.z0 > 0 || ops[i]->mesh.z0 + ops[i]->nc[2] < ops[i]->mesh.nzg) {
            set_error("sipg_batch_create: entry " + std::to_string(i) + " is a slab with neighbours");
            return SIPG_E_ARG;
        }
        if (device >= 0 && ops[i]->device != device) {
            set_error("sipg_batch_create: operators live on different devices");
            return SIPG_E_ARG;
        }
        device = ops[i]->device;
        const size_t bytes = size_t(ops[i]->ndofs) * (ops[i]->dtype == SIPG_F64 ? 8 : 4);
        const char* px = static_cast<const char*>(x[i]);
        const char* py = static_cast<const char*>(y[i]);
        ranges.push_back({px, px + bytes, i, false});
        ranges.push_back({py, py + bytes, i, true});
    }
    std::string why;
    if (ranges_conflict(ranges, why)) { set_error("sipg_batch_create: " + why); return SIPG_E_ARG; }

    // group by (n, basis, dtype, kernel geometry variant); std::map gives a fixed order
    std::map<std::tuple<int, int, int, int>, std::vector<int>> by_key;
    for (int i = 0; i < nops; ++i)
        by_key[{ops[i]->n, ops[i]->basis, ops[i]->dtype, matvec_geom(ops[i])}].push_back(i);

    auto* b = new (std::nothrow) sipg_batch;
    if (!b) { set_error("sipg_batch_create: out of host memory"); return SIPG_E_OOM; }
    b->device = device;
    b->nops = nops;
    b->ops.assign(ops, ops + nops);
    b->x.assign(x, x + nops);
    b->y.assign(y, y + nops);
    // host images of the device arrays, laid out group after group
    std::vector<char> host;
    struct Off { size_t params, blk_op, blk_first; };
    std::vector<Off> offs;
    for (const auto& kv : by_key) {
        const auto [n, basis, dtype, geom] = kv.first;
        const std::vector<int>& idx = kv.second;
        const int cpb = cells_per_block(n);
        BatchGroup g;
        g.n = n; g.basis = basis; g.dtype = dtype; g.geom = geom;
        g.nops = int(idx.size());
        std::vector<int> first(idx.size());
        int64_t nblk = 0;
        for (size_t j = 0; j < idx.size(); ++j) {
            first[j] = int(nblk);
            nblk += (ops[idx[j]]->ncells + cpb - 1) / cpb;
            g.ndofs += ops[idx[j]]->ndofs;
            b->ncells += ops[idx[j]]->ncells;
        }
        if (nblk >= (int64_t(1) << 31)) {
            delete b;
            set_error("sipg_batch_create: a group exceeds 2^31 workgroups");
            return SIPG_E_ARG;
        }
        g.nblocks = nblk;
        std::vector<int> blk_op(static_cast<size_t>(nblk), 0);
        for (size_t j = 0; j < idx.size(); ++j) {
            const int64_t e = j + 1 < idx.size() ? first[j + 1] : nblk;
            std::fill(blk_op.begin() + first[j], blk_op.begin() + e, int(j));
        }
        const size_t psz = sizeof(MatvecParams<double>) * idx.size();
        static_assert(sizeof(MatvecParams<double>) == sizeof(MatvecParams<float>), "same parameter layout");
        Off o;
        o.params = align_up(host.size());
        o.blk_first = align_up(o.params + psz);
        o.blk_op = align_up(o.blk_first + sizeof(int) * first.size());
        host.resize(align_up(o.blk_op + sizeof(int) * blk_op.size()));
        for (size_t j = 0; j < idx.size(); ++j) {
            const int i = idx[j];
            if (dtype == SIPG_F64) {
                const MatvecParams<double> p = matvec_params<double>(ops[i], x[i], y[i]);
                std::memcpy(host.data() + o.params + j * sizeof(p), &p, sizeof(p));
            } else {
                const MatvecParams<float> p = matvec_params<float>(ops[i], x[i], y[i]);
                std::memcpy(host.data() + o.params + j * sizeof(p), &p, sizeof(p));
            }
        }
        std::memcpy(host.data() + o.blk_first, first.data(), sizeof(int) * first.size());
        std::memcpy(host.data() + o.blk_op, blk_op.data(), sizeof(int) * blk_op.size());
        offs.push_back(o);
        b->ndofs += g.ndofs;
        b->nblocks += nblk;
        b->groups.push_back(g);
        b->members.push_back(idx);
        b->schedule.push_back(0);
    }
    int prev = 0;
    (void)hipGetDevice(&prev);
    // the table comes from the allocator of the first operator
    b->alloc = ops[0]->mem;
    hipError_t e = hipSetDevice(device);
    int arc = SIPG_OK;
    if (e == hipSuccess) arc = b->alloc.alloc(&b->mem, host.size(), "sipg_batch_create: device tables");
    if (e == hipSuccess && arc == SIPG_OK) e = hipMemcpy(b->mem, host.data(), host.size(), hipMemcpyHostToDevice);
    (void)hipSetDevice(prev);
    if (e != hipSuccess || arc != SIPG_OK) {
        b->alloc.release(b->mem);
        delete b;
        return arc != SIPG_OK ? arc : hip_fail(e, "sipg_batch_create: device tables");
    }
    b->bytes = host.size();
    // groups to streams: largest first, each to the stream with the fewest
    // workgroups so far (at most 4 streams: the device's hardware queues)
    {
        const int nlanes = int(std::min<size_t>(4, b->groups.size()));
        std::vector<size_t> idx(b->groups.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
        std::sort(idx.begin(), idx.end(), [&](size_t a, size_t c) { return b->groups[a].nblocks > b->groups[c].nblocks; });
        std::vector<int64_t> load(nlanes, 0);
        b->lane.assign(b->groups.size(), 0);
        for (size_t i : idx) {
            const int l = int(std::min_element(load.begin(), load.end()) - load.begin());
            b->lane[i] = l;
            load[l] += b->groups[i].nblocks;
        }
        (void)hipGetDevice(&prev);
        hipError_t se = hipSetDevice(device);
        if (se == hipSuccess) se = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        for (int l = 1; l < nlanes && se == hipSuccess; ++l) {
            hipStream_t s2 = nullptr;
            hipEvent_t ev = nullptr;
            se = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
            if (se == hipSuccess) b->aux.push_back(s2);
            if (se == hipSuccess) se = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (se == hipSuccess) b->join.push_back(ev);
        }
        (void)hipSetDevice(prev);
        if (se != hipSuccess) {
            sipg_batch_destroy(b);
            return hip_fail(se, "sipg_batch_create: streams");
        }
    }
    char* base = static_cast<char*>(b->mem);
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        b->groups[gi].params = base + offs[gi].params;
        b->groups[gi].blk_first = reinterpret_cast<const int*>(base + offs[gi].blk_first);
        b->groups[gi].blk_op = reinterpret_cast<const int*>(base + offs[gi].blk_op);
    }
    *out = b;
    return SIPG_OK;
}

static int run_group(const sipg_batch* b, size_t gi, int schedule, hipStream_t st) {
    if (schedule == 0) return launch_matvec_batched(b->groups[gi], st);
    for (int i : b->members[gi])
        if (int rc = launch_matvec(b->ops[i], b->x[i], b->y[i], st)) return rc;
    return SIPG_OK;
}

int sipg_batch_apply(const sipg_batch* b, void* stream) {
    if (!b) { set_error("sipg_batch_apply: null batch"); return SIPG_E_ARG; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the aux streams start after the work queued on the caller's stream
    SIPG_HIP(hipEventRecord(b->fork, st));
    for (hipStream_t s2 : b->aux) SIPG_HIP(hipStreamWaitEvent(s2, b->fork, 0));
    int rc = SIPG_OK;
    for (size_t gi = 0; gi < b->groups.size() && rc == SIPG_OK; ++gi)
        rc = run_group(b, gi, b->schedule[gi], b->lane[gi] == 0 ? st : b->aux[b->lane[gi] - 1]);
    // and the caller's stream continues after all of them (also on error, so
    // that nothing queued later overtakes a launched group)
    for (size_t j = 0; j < b->aux.size(); ++j) {
        SIPG_HIP(hipEventRecord(b->join[j], b->aux[j]));
        SIPG_HIP(hipStreamWaitEvent(st, b->join[j], 0));
    }
    return rc;
}

int sipg_batch_tune(sipg_batch* b, int reps, void* stream) {
    if (!b || reps < 1) { set_error("sipg_batch_tune: null batch or reps < 1"); return SIPG_E_ARG; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    SIPG_HIP(hipEventCreate(&e0));
    SIPG_HIP(hipEventCreate(&e1));
    int rc = SIPG_OK;
    for (size_t gi = 0; gi < b->groups.size() && rc == SIPG_OK; ++gi) {
        float best = 0.0f;
        int pick = 0;
        for (int sched = 0; sched < 2 && rc == SIPG_OK; ++sched) {
            if ((rc = run_group(b, gi, sched, st)) != SIPG_OK) break;   // warm-up
            hipError_t e = hipEventRecord(e0, st);
            for (int r = 0; r < reps && rc == SIPG_OK && e == hipSuccess; ++r) rc = run_group(b, gi, sched, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) { rc = hip_fail(e, "sipg_batch_tune: timing"); break; }
            if (sched == 0 || ms < best) { best = ms; pick = sched; }
        }
        b->schedule[gi] = pick;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int sipg_batch_get_info(const sipg_batch* b, sipg_batch_info* info) {
    if (!b || !info) { set_error("sipg_batch_get_info: null argument"); return SIPG_E_ARG; }
    info->nops = b->nops;
    info->launches = int(b->groups.size());
    info->ndofs = b->ndofs;
    info->ncells = b->ncells;
    info->workgroups = b->nblocks;
    info->device_bytes = int64_t(b->bytes);
    info->per_operator_groups = 0;
    for (int sch : b->schedule) info->per_operator_groups += sch;
    info->streams = int32_t(b->aux.size()) + 1;
    return SIPG_OK;
}

int sipg_batch_destroy(sipg_batch* b) {
    if (!b) return SIPG_OK;
    b->alloc.release(b->mem);
    for (hipStream_t s2 : b->aux) (void)hipStreamDestroy(s2);
    for (hipEvent_t ev : b->join) (void)hipEventDestroy(ev);
    if (b->fork) (void)hipEventDestroy(b->fork);
    delete b;
    return SIPG_OK;
}

}  // extern "C"
