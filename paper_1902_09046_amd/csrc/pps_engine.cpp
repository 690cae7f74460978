// Epoch engine (see pps_engine.hpp).
#include "pps_engine.hpp"

#include <chrono>
#include <cstring>

#include "pps_runtime.hpp"

namespace pps {

static hipError_t host_alloc(void **p, size_t bytes)
{
    // Coherent mapped host memory: the device reads the tables the host wrote
    // for this epoch (never a cached copy of a previous epoch) and writes the
    // results where the host reads them after the epoch's event.
    hipError_t e = hipHostMalloc(p, bytes, hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess)
        std::memset(*p, 0, bytes);
    return e;
}

template <class T> static T *dev_view(T *host)
{
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, host, 0) != hipSuccess)
        return nullptr;
    return static_cast<T *>(d);
}

EpochEngine::~EpochEngine()
{
    // every epoch ends before anything is freed (an epoch on one slot's
    // stream may wait on another slot's event)
    for (Slot &s : slots_)
        if (s.in_flight && s.done)
            (void)hipEventSynchronize(s.done);
    for (Slot &s : slots_) {
        for (auto &kv : s.execs)
            (void)hipGraphExecDestroy(kv.second);
        for (void *h : {static_cast<void *>(s.h_hdr), static_cast<void *>(s.h_rows),
                        static_cast<void *>(s.h_fins), static_cast<void *>(s.h_out_fin),
                        static_cast<void *>(s.h_out_counts)})
            if (h)
                (void)hipHostFree(h);
        for (void *d : {static_cast<void *>(s.dev.d_hdr), static_cast<void *>(s.dev.d_rows),
                        static_cast<void *>(s.dev.d_fins), static_cast<void *>(s.dev.states)})
            if (d)
                (void)hipFree(d);
        for (hipEvent_t ev : {s.sim_start, s.sim_stop, s.fin_stop, s.done})
            if (ev)
                (void)hipEventDestroy(ev);
        if (s.own_stream)
            (void)hipStreamDestroy(s.own_stream);
    }
    if (capture_stream_)
        (void)hipStreamDestroy(capture_stream_);
}

int EpochEngine::init(int n_slots, int cu_count)
{
    cu_count_ = cu_count;
    // The cell kernel holds 32 KB of LDS per workgroup: 512 lanes per
    // workgroup reach 8 waves per SIMD, 256 would stop at 5.
    shape_.sim[CLASS_CELLS].block = 512;
    // One tuberculosis draw per 64-lane workgroup.
    shape_.sim[CLASS_GILLESPIE].block = 64;
    hipError_t e = hipStreamCreateWithFlags(&capture_stream_, hipStreamNonBlocking);
    if (e != hipSuccess)
        return fail_hip(e, "capture stream");
    slots_.resize(n_slots);
    for (Slot &s : slots_) {
        void *p;
        if ((e = host_alloc(&p, sizeof(EpochHeader))) != hipSuccess)
            return fail_hip(e, "epoch header staging");
        s.h_hdr = static_cast<EpochHeader *>(p);
        if ((e = host_alloc(&p, MAX_ROWS * sizeof(JobDev))) != hipSuccess)
            return fail_hip(e, "row staging");
        s.h_rows = static_cast<JobDev *>(p);
        if ((e = host_alloc(&p, MAX_FINS * sizeof(FinJob))) != hipSuccess)
            return fail_hip(e, "finalisation staging");
        s.h_fins = static_cast<FinJob *>(p);
        if ((e = host_alloc(&p, MAX_FINS * sizeof(FinResult))) != hipSuccess)
            return fail_hip(e, "result staging");
        s.h_out_fin = static_cast<FinResult *>(p);
        if ((e = host_alloc(&p, MAX_OUT_COUNTS * sizeof(unsigned long long))) != hipSuccess)
            return fail_hip(e, "count staging");
        s.h_out_counts = static_cast<unsigned long long *>(p);
        s.dev.h_hdr = dev_view(s.h_hdr);
        s.dev.h_rows = dev_view(s.h_rows);
        s.dev.h_fins = dev_view(s.h_fins);
        s.dev.h_out_fin = dev_view(s.h_out_fin);
        s.dev.h_out_counts = dev_view(s.h_out_counts);
        if (!s.dev.h_hdr || !s.dev.h_rows || !s.dev.h_fins || !s.dev.h_out_fin || !s.dev.h_out_counts)
            return fail(PPS_EDEVICE, "mapped staging has no device address");
        if ((e = hipMalloc(&p, sizeof(EpochHeader))) != hipSuccess)
            return fail_hip(e, "device epoch header");
        s.dev.d_hdr = static_cast<EpochHeader *>(p);
        if ((e = hipMalloc(&p, MAX_ROWS * sizeof(JobDev))) != hipSuccess)
            return fail_hip(e, "device row table");
        s.dev.d_rows = static_cast<JobDev *>(p);
        if ((e = hipMalloc(&p, MAX_FINS * sizeof(FinJob))) != hipSuccess)
            return fail_hip(e, "device finalisation table");
        s.dev.d_fins = static_cast<FinJob *>(p);
        if ((e = hipMalloc(&p, N_CLASSES * sizeof(LaunchState))) != hipSuccess)
            return fail_hip(e, "launch state");
        s.dev.states = static_cast<LaunchState *>(p);
        if ((e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreate(&s.sim_start)) != hipSuccess ||
            (e = hipEventCreate(&s.sim_stop)) != hipSuccess ||
            (e = hipEventCreate(&s.fin_stop)) != hipSuccess)
            return fail_hip(e, "epoch events");
        if (&s != &slots_[0] &&
            (e = hipStreamCreateWithFlags(&s.own_stream, hipStreamNonBlocking)) != hipSuccess)
            return fail_hip(e, "epoch stream");
    }
    return PPS_OK;
}

int EpochEngine::set_graph_shape(Slot &s, bool build)
{
    EpochShape want = shape_;
    for (int c = 0; c < N_CLASSES; ++c) {
        if (!sim_shape_supported(c, want.sim[c]))
            return fail(PPS_EINVAL, "unsupported launch shape for class %d", c);
        int per_cu = 0;
        hipError_t e = sim_occupancy(c, want.sim[c], &per_cu);
        if (e != hipSuccess || per_cu < 1)
            per_cu = 1;
        want.sim_grid[c] = static_cast<unsigned>(per_cu * cu_count_);
    }
    want.fin_grid = static_cast<unsigned>(8 * cu_count_);
    if (s.have_shape && s.exec_shape == want)
        return PPS_OK;
    if (!build)
        return fail(PPS_EINVAL, "the launch shape changed since the epoch graphs were built");
    for (auto &kv : s.execs)
        (void)hipGraphExecDestroy(kv.second);
    s.execs.clear();
    s.exec_shape = want;
    s.have_shape = true;
    return PPS_OK;
}

// Adds a record of `ev` after everything captured so far on `cs` and makes
// the work captured next follow it.  (An event recorded on a capturing stream
// is not turned into a graph node by this runtime, so the node is added
// explicitly.)
static hipError_t capture_event(hipStream_t cs, hipEvent_t ev)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    unsigned long long id = 0;
    hipGraph_t g = nullptr;
    const hipGraphNode_t *deps = nullptr;
    size_t n_deps = 0;
    hipError_t e = hipStreamGetCaptureInfo_v2(cs, &st, &id, &g, &deps, &n_deps);
    if (e != hipSuccess)
        return e;
    if (st != hipStreamCaptureStatusActive || !g)
        return hipErrorStreamCaptureInvalidated;
    hipGraphNode_t node = nullptr;
    e = hipGraphAddEventRecordNode(&node, g, deps, n_deps, ev);
    if (e != hipSuccess)
        return e;
    return hipStreamUpdateCaptureDependencies(cs, &node, 1, hipStreamSetCaptureDependencies);
}

// Form bits: bit c = class c has tiles; bits N_CLASSES.. = 0 no
// finalisation, 1 with the selection passes, 2 fixed tolerances only.
int EpochEngine::graph_for(Slot &s, unsigned form, hipGraphExec_t *out, bool build)
{
    auto it = s.execs.find(form);
    if (it != s.execs.end()) {
        *out = it->second;
        return PPS_OK;
    }
    if (!build)
        return fail(PPS_EINVAL, "no epoch graph of this form has been built on the device yet");
    const EpochShape &sh = s.exec_shape;
    hipError_t e = hipStreamBeginCapture(capture_stream_, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return fail_hip(e, "graph capture begin");
    // stage-in, [sim_start], the simulation of each class with tiles,
    // [sim_stop], the finalisation, stage-out
    hipError_t ei = issue_epoch_part(EPOCH_STAGE_IN, s.dev, sh, capture_stream_);
    if (ei == hipSuccess)
        ei = capture_event(capture_stream_, s.sim_start);
    for (int c = 0; c < N_CLASSES && ei == hipSuccess; ++c)
        if (form & (1u << c))
            ei = issue_epoch_part(EPOCH_SIMULATE + c, s.dev, sh, capture_stream_);
    if (ei == hipSuccess)
        ei = capture_event(capture_stream_, s.sim_stop);
    const unsigned fin = form >> N_CLASSES;
    if (ei == hipSuccess && fin != 0)
        ei = issue_epoch_part(fin == 1 ? EPOCH_FINALIZE : EPOCH_FINALIZE_FIXED, s.dev, sh,
                              capture_stream_);
    if (ei == hipSuccess && fin != 0)
        ei = capture_event(capture_stream_, s.fin_stop);
    if (ei == hipSuccess)
        ei = issue_epoch_part(EPOCH_STAGE_OUT, s.dev, sh, capture_stream_);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(capture_stream_, &graph);
    if (ei != hipSuccess || e != hipSuccess) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return fail_hip(ei != hipSuccess ? ei : e, "epoch capture");
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess)
        return fail_hip(e, "graph instantiate");
    s.execs[form] = x;
    *out = x;
    return PPS_OK;
}

int EpochEngine::launch(int slot, EpochPlan &plan, hipStream_t stream, bool build)
{
    Slot &s = slots_[slot];
    if (s.in_flight)
        return fail(PPS_EBUSY, "epoch slot %d still in flight", slot);
    size_t n_rows = 0;
    for (int c = 0; c < N_CLASSES; ++c)
        n_rows += plan.rows[c].size();
    if (n_rows > static_cast<size_t>(MAX_ROWS) || plan.fins.size() > static_cast<size_t>(MAX_FINS))
        return fail(PPS_EINVAL, "epoch too large: %zu rows, %zu finalisations", n_rows,
                    plan.fins.size());
    int rc = set_graph_shape(s, build);
    if (rc != PPS_OK)
        return rc;
    EpochHeader &H = *s.h_hdr;
    std::memset(&H, 0, sizeof H);
    uint32_t r = 0;
    uint32_t out_slot = 0;
    for (int c = 0; c < N_CLASSES; ++c) {
        H.class_first[c] = r;
        H.class_rows[c] = static_cast<uint32_t>(plan.rows[c].size());
        uint64_t tiles = 0;
        const uint64_t ts = tile_size(c);
        if (c == CLASS_GROUP && plan.rows[c].size() % GROUP_LPL != 0)
            return fail(PPS_EINVAL, "lambda-group rows must come in groups of %d", GROUP_LPL);
        for (size_t i = 0; i < plan.rows[c].size(); ++i) {
            JobDev &row = plan.rows[c][i];
            row.tile_size = static_cast<int32_t>(ts);
            row.tile_begin = tiles;
            // the members of a lambda group share the group's tiles
            if (c != CLASS_GROUP || i % GROUP_LPL == GROUP_LPL - 1)
                tiles += row.n_tiles;
            if (row.row_flags & ROW_COPY_COUNTS) {
                if (out_slot + row.n_counts > static_cast<uint32_t>(MAX_OUT_COUNTS))
                    return fail(PPS_EINVAL, "epoch has too many tallies");
                row.out_slot = out_slot;
                out_slot += row.n_counts;
            }
            s.h_rows[r++] = row;
        }
        H.class_tiles[c] = tiles;
    }
    H.n_rows = r;
    uint64_t fb = 0;
    for (size_t i = 0; i < plan.fins.size(); ++i) {
        FinJob &F = plan.fins[i];
        F.n_blocks = (F.n + FIN_TILE - 1) / FIN_TILE;
        F.block_begin = fb;
        fb += F.n_blocks;
        if (F.mode == PPS_EPS_TOP_FRACTION)
            H.any_top = 1;
        s.h_fins[i] = F;
    }
    H.n_fins = static_cast<uint32_t>(plan.fins.size());
    H.fin_blocks = fb;
    unsigned form = 0;
    for (int c = 0; c < N_CLASSES; ++c)
        if (H.class_tiles[c] > 0)
            form |= 1u << c;
    if (H.n_fins > 0)
        form |= (H.any_top ? 1u : 2u) << N_CLASSES;
    hipGraphExec_t x = nullptr;
    if ((rc = graph_for(s, form, &x, build)) != PPS_OK)
        return rc;
    hipError_t e = hipSuccess;
    if (last_slot_ >= 0 && last_stream_ != stream)
        e = hipStreamWaitEvent(stream, slots_[last_slot_].sim_stop, 0);
    if (e == hipSuccess)
        e = hipGraphLaunch(x, stream);
    if (e != hipSuccess)
        return fail_hip(e, "epoch graph launch");
    e = hipEventRecord(s.done, stream);
    if (e != hipSuccess)
        return fail_hip(e, "epoch event");
    s.in_flight = true;
    s.has_fin = H.n_fins > 0;
    last_slot_ = slot;
    last_stream_ = stream;
    return PPS_OK;
}

int EpochEngine::finish(Slot &s)
{
    s.in_flight = false;
    float ms = -1.0f;
    if (hipEventElapsedTime(&ms, s.sim_start, s.sim_stop) != hipSuccess) {
        (void)hipGetLastError();
        ms = -1.0f;
    }
    s.sim_ms = ms;
    float fms = -1.0f;
    if (s.has_fin && hipEventElapsedTime(&fms, s.sim_stop, s.fin_stop) != hipSuccess) {
        (void)hipGetLastError();
        fms = -1.0f;
    }
    s.fin_ms = s.has_fin ? fms : -1.0f;
    return PPS_OK;
}

int EpochEngine::wait(int slot)
{
    Slot &s = slots_[slot];
    if (!s.in_flight)
        return PPS_OK;
    // poll the completion event (the caller waits on this thread anyway);
    // hand over to the runtime's blocking wait after a long epoch
    hipError_t e = hipErrorNotReady;
    const auto t0 = std::chrono::steady_clock::now();
    while ((e = hipEventQuery(s.done)) == hipErrorNotReady &&
           std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(50)) {
    }
    if (e == hipErrorNotReady)
        e = hipEventSynchronize(s.done);
    if (e != hipSuccess) {
        s.in_flight = false;
        return fail_hip(e, "epoch");
    }
    return finish(s);
}

int EpochEngine::poll(int slot)
{
    Slot &s = slots_[slot];
    if (!s.in_flight)
        return PPS_OK;
    hipError_t e = hipEventQuery(s.done);
    if (e == hipErrorNotReady)
        return PPS_PENDING;
    if (e != hipSuccess) {
        s.in_flight = false;
        return fail_hip(e, "epoch");
    }
    return finish(s);
}

}  // namespace pps
