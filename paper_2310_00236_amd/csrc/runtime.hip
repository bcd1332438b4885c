// Host runtime behind the C ABI of halfwave.h: problem validation, arena
// carving, uploads and downloads, the time loop, the energy trace,
// checkpoints and batched launches over many plans.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "halfwave.h"
#include "hw_internal.h"

using namespace hw;

// Device memory of hw_simulate_noalloc: one copy per GPU, held from the
// module's load on that GPU until the process ends.  Host code never uses
// this name as an address; it goes through scratch_address().
static __device__ __align__(256) unsigned char scratch[HW_NOALLOC_MAX_BYTES];

namespace {

thread_local std::string g_error;

hw_status fail(hw_status st, const std::string &msg)
{
    g_error = msg;
    return st;
}

#define HW_HIP(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess)                                                 \
            return fail(HW_E_DEVICE, std::string(#call ": ") +                \
                                         hipGetErrorString(e_));              \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int32_t kMaxReceivers = 64;
constexpr int64_t kPitchAlign = 64;   // elements

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int esize(int storage) { return storage == HW_F32 ? 4 : 2; }

double max_finite(int storage)
{
    switch (storage) {
    case HW_F16: return 65504.0;
    case HW_BF16: return 0x1.fep127;
    default: return 0x1.fffffep127;
    }
}

double cfl_bound(int physics, int order)
{
    if (physics == HW_ACOUSTIC2D) {
        if (order == 2)
            return 1.0 / std::sqrt(2.0);
        if (order == 4)
            return 1.0 / (std::sqrt(2.0) * (9.0 / 8.0 + 1.0 / 24.0));
        return -1.0;
    }
    if (physics == HW_ELASTIC3D && order == 2)
        return 1.0 / std::sqrt(3.0);
    if (physics == HW_ELASTIC2D && order == 2)
        return 1.0 / std::sqrt(2.0);
    return -1.0;
}

// Layout of a plan inside its arena.
struct Layout {
    int nf = 0, nm = 0, sets = 1;
    int64_t pitch = 0, slab = 0, rows = 0, cells = 0;
    int words = 1;                 // storage values per cell and field
    bool c8 = false;               // 8-bit compensation words
    size_t comp_off = 0;           // their offset after each value array
    size_t field_bytes = 0, mat_bytes = 0;
    size_t off_fld[2][9] = {};
    size_t off_mat[4] = {}, off_staging = 0, off_partial = 0, off_trace = 0;
    int rec_vals = 3;              // values per receiver and trace row
    size_t off_flags = 0, off_desc = 0, total = 0;
    size_t off_src = 0, off_recxy = 0, off_rec = 0;
};

hw_status validate(const hw_problem *pb)
{
    if (!pb)
        return fail(HW_E_INVAL, "problem is NULL");
    if (pb->abi_version != HW_ABI_VERSION)
        return fail(HW_E_INVAL, "abi_version mismatch");
    if (pb->physics != HW_ACOUSTIC2D && pb->physics != HW_ELASTIC3D &&
        pb->physics != HW_ELASTIC2D)
        return fail(HW_E_INVAL, "unknown physics");
    if (cfl_bound(pb->physics, pb->order) < 0)
        return fail(HW_E_INVAL, "unsupported order for this physics");
    if (pb->storage < HW_F32 || pb->storage > HW_BF16)
        return fail(HW_E_INVAL, "unknown storage format");
    if (pb->comp < HW_COMP_NONE || pb->comp > HW_COMP_TWOSUM8)
        return fail(HW_E_INVAL, "unknown compensation mode");
    if (pb->comp == HW_COMP_TWOSUM8 &&
        (pb->physics != HW_ACOUSTIC2D || pb->storage == HW_F32))
        return fail(HW_E_INVAL, "8-bit compensation words are for acoustic "
                                "fp16 / bf16 plans");
    if (pb->scale_log2 < -60 || pb->scale_log2 > 60)
        return fail(HW_E_INVAL, "scale_log2 out of [-60, 60]");
    if (pb->nx < 1 || pb->ny < 1 || pb->nz < 1)
        return fail(HW_E_INVAL, "grid sizes must be >= 1");
    if (pb->physics != HW_ELASTIC3D && pb->nz != 1)
        return fail(HW_E_INVAL, "nz must be 1 for 2D problems");
    if (pb->physics == HW_ELASTIC2D && pb->ny < 3)
        return fail(HW_E_INVAL, "elastic2d needs ny >= 3 (two free surfaces "
                                "and an interior row)");
    const double lim = 1u << 30;
    if ((double)pb->nx > lim || (double)pb->ny > lim || (double)pb->nz > lim ||
        (double)pb->nx * pb->ny * pb->nz > 0x1p40)
        return fail(HW_E_INVAL, "grid too large");
    if (!(pb->dx > 0) || !std::isfinite(pb->dx) || !(pb->dt > 0) ||
        !std::isfinite(pb->dt))
        return fail(HW_E_INVAL, "dx and dt must be finite and > 0");
    if (pb->trace_cap < 0)
        return fail(HW_E_INVAL, "trace_cap must be >= 0");
    if (pb->src_cap < 0 || pb->rec_cap < 0 || pb->rec_cap > kMaxReceivers ||
        pb->rec_steps < 0)
        return fail(HW_E_INVAL, "src_cap, rec_steps must be >= 0, rec_cap in "
                                "[0, 64]");
    if (pb->stencil < HW_STENCIL_F32 || pb->stencil > HW_STENCIL_F64)
        return fail(HW_E_INVAL, "unknown stencil precision");
    if (pb->physics == HW_ELASTIC3D &&
        (pb->src_cap != 0 || pb->rec_cap != 0 || pb->rec_steps != 0))
        return fail(HW_E_INVAL, "sources and receivers are 2D only");
    if (pb->physics != HW_ACOUSTIC2D && pb->stencil != HW_STENCIL_F32)
        return fail(HW_E_INVAL, "stencil precisions are acoustic only");
    if ((double)pb->src_cap > 0x1p40 ||
        (double)pb->rec_steps * (double)pb->rec_cap > 0x1p36)
        return fail(HW_E_INVAL, "source or receiver capacity too large");
    const float w = (float)(pb->dt / pb->dx);
    if (!std::isfinite(w) || w == 0.0f)
        return fail(HW_E_INVAL, "dt/dx does not fit fp32");
    // kernels index each array with 32-bit offsets (padded rows)
    const double padded = std::ceil(pb->nx / (double)kPitchAlign) * kPitchAlign *
                          (double)pb->ny * (double)pb->nz;
    if (padded > 2147483647.0)
        return fail(HW_E_INVAL, "grid too large for 32-bit indexing (padded "
                                "nx*ny*nz must stay below 2^31)");
    return HW_OK;
}

Layout make_layout(const hw_problem *pb)
{
    Layout L;
    const bool ac = pb->physics == HW_ACOUSTIC2D;
    const bool el2 = pb->physics == HW_ELASTIC2D;
    L.nf = ac ? 3 : el2 ? 5 : 9;
    // device material arrays (2D elastic: the four per-cell coefficients)
    L.nm = ac ? 2 : el2 ? 4 : 3;
    L.rec_vals = el2 ? 5 : 3;
    L.sets = 2;
    L.pitch = (pb->nx + kPitchAlign - 1) / kPitchAlign * kPitchAlign;
    L.slab = L.pitch * pb->ny;
    L.rows = pb->ny * pb->nz;
    L.cells = pb->nx * pb->ny * pb->nz;
    // with compensation each cell holds (value, compensation) side by side
    // 8-bit compensation words: a byte array after each value array
    L.c8 = pb->comp == HW_COMP_TWOSUM8;
    L.words = pb->comp != HW_COMP_NONE && !L.c8 ? 2 : 1;
    L.comp_off = L.c8 ? (size_t)(L.slab * pb->nz) * esize(pb->storage) : 0;
    L.field_bytes = align_up((size_t)(L.slab * pb->nz) * esize(pb->storage) * L.words +
                                 (L.c8 ? (size_t)(L.slab * pb->nz) : 0),
                             kAlign);
    L.mat_bytes = align_up((size_t)(L.slab * pb->nz) * 4, kAlign);
    size_t off = 0;
    for (int s = 0; s < L.sets; ++s)
        for (int f = 0; f < L.nf; ++f) {
            L.off_fld[s][f] = off;
            off += L.field_bytes;
        }
    for (int m = 0; m < L.nm; ++m) {
        L.off_mat[m] = off;
        off += L.mat_bytes;
    }
    L.off_staging = off;
    off += align_up((size_t)L.cells * 8, kAlign);
    L.off_partial = off;
    off += align_up((size_t)L.rows * 8, kAlign);
    L.off_trace = off;
    off += align_up((size_t)std::max<int64_t>(pb->trace_cap, 1) * 8, kAlign);
    L.off_flags = off;             // status flag (int32) and step counter (int64 at +8)
    off += kAlign;
    L.off_src = off;
    off += align_up((size_t)pb->src_cap * 4, kAlign);
    L.off_recxy = off;
    off += align_up((size_t)pb->rec_cap * 8, kAlign);
    L.off_rec = off;
    off += align_up((size_t)pb->rec_steps * pb->rec_cap * L.rec_vals * 8, kAlign);
    L.off_desc = off;
    off += align_up(std::max({sizeof(Ac2dDesc), sizeof(El3dDesc), sizeof(El2dDesc)}),
                    kAlign);
    L.total = off;
    return L;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the calling thread's current device,
// looked up once per device (each GPU holds its own copy at its own
// address).
hw_status scratch_address(void **out)
{
    int dev = 0;
    HW_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(HW_E_DEVICE, "device index " + std::to_string(dev) + " beyond " +
                                     std::to_string(kMaxDevices));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HW_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || (uintptr_t)ptr % kAlign != 0)
            return fail(HW_E_DEVICE, "scratch array has no aligned device address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HW_OK;
}

struct KernelKey {
    int physics, order, storage, comp, stencil;
    bool operator<(const KernelKey &o) const
    {
        return std::tie(physics, order, storage, comp, stencil) <
               std::tie(o.physics, o.order, o.storage, o.comp, o.stencil);
    }
};

}  // namespace

struct hw_plan {
    hw_problem pb;
    Layout L;
    char *arena;
    void *fld[2][9];
    float *mat[4];
    double *staging, *partial, *trace;
    int32_t *flags;
    void *d_desc;
    Ac2dDesc h2;
    El3dDesc h3;
    El2dDesc he;
    int cur = 0;
    int64_t step = 0;
    int64_t trace_n = 0;
    int64_t last_logged = -1;
    std::vector<int64_t> trace_steps;
    bool have_material = false, have_fields = false;
    int tile = 0;
    double scale_up = 1.0, scale_down = 1.0;
    int64_t *counter = nullptr;    // device step counter (sources, receivers)
    bool counts() const
    {
        return pb.physics == HW_ELASTIC2D ? he.src_n > 0 || he.rec_n > 0
                                          : h2.src_n > 0 || h2.rec_n > 0;
    }
    // captured run of kGraphSteps steps starting from field set 0
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    int graph_tile = -1;
    // launch every step directly: no capture stream, no graph (the
    // no-allocation entry point creates no runtime objects)
    bool direct = false;
    KernelKey key() const { return {pb.physics, pb.order, pb.storage, pb.comp, pb.stencil}; }
    ~hw_plan()
    {
        if (graph)
            (void)hipGraphExecDestroy(graph);
        if (cap_stream)
            (void)hipStreamDestroy(cap_stream);
    }
};

namespace {

hipStream_t S(void *s) { return (hipStream_t)s; }

const TileShape *tile_table(int physics)
{
    return physics == HW_ACOUSTIC2D ? kTiles2D : physics == HW_ELASTIC3D ? kTiles3D
                                                                           : kTilesEl2D;
}

int tile_count(int physics)
{
    return physics == HW_ACOUSTIC2D ? kNumTiles2D
           : physics == HW_ELASTIC3D ? kNumTiles3D
           : physics == HW_ELASTIC2D ? kNumTilesEl2D
                                     : 0;
}

int num_tiles(const hw_problem &pb) { return tile_count(pb.physics); }

void tile_counts(const hw_plan *p, int tile, int32_t *tx, int32_t *ty, int32_t *total)
{
    const TileShape t = tile_table(p->pb.physics)[tile];
    *tx = (int32_t)((p->pb.nx + t.tx - 1) / t.tx);
    *ty = (int32_t)((p->pb.ny + t.ty - 1) / t.ty);
    *total = *tx * *ty * (int32_t)((p->pb.nz + t.tz - 1) / t.tz);
}

// Steps launched between host interventions are captured into a HIP graph
// in runs of this many (a multiple of 4: an even number of launches of one
// or two steps, so every shot's field set returns to where the run started).
constexpr int kGraphSteps = 32;
static_assert(kGraphSteps % 4 == 0, "graph runs of an even number of launches");

// The shape a group of plans sharing a kernel runs on when given `tile`:
// acoustic plans with a point source or receivers or a non-default stencil
// run on shape 0, 8-bit compensation words on any shape but the marching
// kind 1 (else shape 0), and `single` asks for a one-step shape (shape 0 in
// place of a two-step one).
int group_tile(hw_plan *const *plans, int n, int tile, bool single)
{
    const hw_plan *p0 = plans[0];
    if (p0->pb.physics != HW_ACOUSTIC2D)
        return tile;
    bool forced = false;
    for (int i = 0; i < n; ++i)
        forced = forced || plans[i]->counts();
    const int kind = kTiles2D[tile].kind;
    const bool two = steps_per_launch2d(kTiles2D[tile]) == 2;
    if (p0->pb.stencil != HW_STENCIL_F32)
        return 0;
    if (single && two)
        return 0;
    // plans with a point source or receivers: the two-step kernels, or the
    // one-step variant kernels of shape 0
    if (forced)
        return two ? tile : 0;
    if (p0->pb.comp == HW_COMP_TWOSUM8 && kind == 1)
        return 0;
    return tile;
}

// Time steps one launch of the group advances on `tile`.
int group_steps(hw_plan *const *plans, int n, int tile)
{
    if (plans[0]->pb.physics != HW_ACOUSTIC2D)
        return 1;
    return steps_per_launch2d(kTiles2D[group_tile(plans, n, tile, false)]);
}

// Launch one launch's worth of time steps (group_steps, or one step if
// `single`) for a group of plans sharing a kernel, in launches of at most
// kMaxBatch shots; parity[i] is plan i's current field set.  Host state is
// not touched (the same launches can be recorded into a graph).
hw_status launch_group_raw(hw_plan *const *plans, int n, int tile,
                           const int *parity, hipStream_t s, bool single = false)
{
    const hw_plan *p0 = plans[0];
    if (p0->pb.physics == HW_ELASTIC2D) {
        // one launch pair per plan (descriptor by value); the plans with a
        // source or receivers count their steps on the device afterwards
        StepCounters c;
        c.n = 0;
        for (int i = 0; i < n; ++i) {
            hw_plan *p = plans[i];
            hipError_t e = launch_el2d_step(p->he, parity[i], p->pb.storage, p->pb.comp,
                                            p->counts(), tile, s);
            if (e == hipSuccess && p->counts()) {
                c.c[c.n++] = p->counter;
                if (c.n == kMaxBatch) {
                    e = launch_tick(c, s);
                    c.n = 0;
                }
            }
            if (e != hipSuccess)
                return fail(HW_E_DEVICE, std::string("step launch: ") + hipGetErrorString(e));
        }
        if (c.n > 0) {
            hipError_t e = launch_tick(c, s);
            if (e != hipSuccess)
                return fail(HW_E_DEVICE, std::string("step launch: ") + hipGetErrorString(e));
        }
        return HW_OK;
    }
    for (int base = 0; base < n; base += kMaxBatch) {
        const int m = std::min(kMaxBatch, n - base);
        hipError_t e;
        if (p0->pb.physics == HW_ACOUSTIC2D) {
            Ac2dBatch a;
            std::memset(&a, 0, sizeof(a));
            a.nshots = m;
            bool forced = false;
            for (int i = 0; i < m; ++i)
                forced = forced || plans[base + i]->counts();
            const int stencil = p0->pb.stencil;
            const int t = group_tile(plans + base, m, tile, single);
            int64_t total = 0;
            for (int i = 0; i < m; ++i) {
                hw_plan *p = plans[base + i];
                int32_t tx, ty, tt;
                tile_counts(p, t, &tx, &ty, &tt);
                a.tile_start[i] = (int32_t)total;
                a.tiles_x[i] = tx;
                a.tiles_y[i] = ty;
                a.parity[i] = parity[base + i];
                a.desc[i] = (const Ac2dDesc *)p->d_desc;
                total += tt;
            }
            if (total > INT32_MAX)
                return fail(HW_E_INVAL, "batch has too many tiles for one launch");
            a.tile_start[m] = (int32_t)total;
            a.total_tiles = (int32_t)total;
            if (steps_per_launch2d(kTiles2D[t]) == 2)
                e = launch_ac2d_step2(a, m == 1 ? &plans[base]->h2 : nullptr,
                                      p0->pb.storage, p0->pb.comp, p0->pb.order, t, forced,
                                      s);
            else
                e = launch_ac2d_step(a, m == 1 ? &plans[base]->h2 : nullptr,
                                     p0->pb.storage, p0->pb.comp, p0->pb.order, t,
                                     forced, stencil, s);
            // plans with a source or receivers count their steps on the device
            StepCounters c;
            c.n = 0;
            c.by = steps_per_launch2d(kTiles2D[t]);
            for (int i = 0; i < m; ++i)
                if (plans[base + i]->counts())
                    c.c[c.n++] = plans[base + i]->counter;
            if (e == hipSuccess && c.n > 0)
                e = launch_tick(c, s);
        } else {
            El3dBatch a;
            std::memset(&a, 0, sizeof(a));
            a.nshots = m;
            int64_t total = 0;
            for (int i = 0; i < m; ++i) {
                hw_plan *p = plans[base + i];
                int32_t tx, ty, tt;
                tile_counts(p, tile, &tx, &ty, &tt);
                a.tile_start[i] = (int32_t)total;
                a.tiles_x[i] = tx;
                a.tiles_y[i] = ty;
                a.parity[i] = parity[base + i];
                a.desc[i] = (const El3dDesc *)p->d_desc;
                total += tt;
            }
            if (total > INT32_MAX)
                return fail(HW_E_INVAL, "batch has too many tiles for one launch");
            a.tile_start[m] = (int32_t)total;
            a.total_tiles = (int32_t)total;
            e = launch_el3d_step(a, m == 1 ? &plans[base]->h3 : nullptr,
                                 p0->pb.storage, p0->pb.comp, tile, s);
        }
        if (e != hipSuccess)
            return fail(HW_E_DEVICE, std::string("step launch: ") + hipGetErrorString(e));
    }
    return HW_OK;
}

// Every launch reads one field set and writes the other.
void advance_state(hw_plan *const *plans, int n, int64_t steps, int64_t launches)
{
    for (int i = 0; i < n; ++i) {
        hw_plan *p = plans[i];
        p->cur ^= (int)(launches & 1);
        p->step += steps;
    }
}

hw_status launch_group(hw_plan *const *plans, int n, int tile, hipStream_t s,
                       bool single = false)
{
    std::vector<int> par(n);
    for (int i = 0; i < n; ++i)
        par[i] = plans[i]->cur;
    hw_status st = launch_group_raw(plans, n, tile, par.data(), s, single);
    if (st == HW_OK)
        advance_state(plans, n, single ? 1 : group_steps(plans, n, tile), 1);
    return st;
}

// Record kGraphSteps steps of one group (starting from the plans' current
// field sets) into an executable graph, via a capture stream: an even number
// of launches, so every plan's field set returns to where the run started.
hw_status capture_run(hw_plan *const *plans, int n, int tile, hipStream_t cap,
                      hipGraphExec_t *out)
{
    std::vector<int> par(n);
    for (int i = 0; i < n; ++i)
        par[i] = plans[i]->cur;
    const int launches = kGraphSteps / group_steps(plans, n, tile);
    HW_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    hw_status st = HW_OK;
    for (int g = 0; g < launches && st == HW_OK; ++g) {
        st = launch_group_raw(plans, n, tile, par.data(), cap);
        for (int i = 0; i < n; ++i)
            par[i] ^= 1;
    }
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cap, &graph);
    if (st != HW_OK) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess)
        return fail(HW_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess)
        return fail(HW_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return HW_OK;
}

thread_local hipStream_t t_cap_stream = nullptr;

// Batch graphs whose last launch was recorded by an event; destroyed once
// that event has completed (never while a launch may still be pending).
struct RetiredGraph {
    hipGraphExec_t exec;
    hipEvent_t done;
};
thread_local std::vector<RetiredGraph> t_retired;

void reap_graphs(bool wait)
{
    for (size_t i = 0; i < t_retired.size();) {
        RetiredGraph &r = t_retired[i];
        if (wait)
            (void)hipEventSynchronize(r.done);
        if (hipEventQuery(r.done) == hipSuccess) {
            (void)hipGraphExecDestroy(r.exec);
            (void)hipEventDestroy(r.done);
            t_retired[i] = t_retired.back();
            t_retired.pop_back();
        } else {
            ++i;
        }
    }
}

hw_status retire_graph(hipGraphExec_t exec, hipStream_t s)
{
    hipEvent_t ev;
    HW_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HW_HIP(hipEventRecord(ev, s));
    t_retired.push_back({exec, ev});
    if (t_retired.size() > 64)
        reap_graphs(true);
    return HW_OK;
}

hw_status capture_stream(hipStream_t *cs)
{
    if (!*cs)
        HW_HIP(hipStreamCreateWithFlags(cs, hipStreamNonBlocking));
    return HW_OK;
}

// Advance a group of plans by `steps` steps with no host work in between:
// whole runs of kGraphSteps replay a captured graph, the rest are launched
// directly.  A single plan keeps its graph (captured from field set 0).
// Direct plans launch every step on `s`.
hw_status run_steps(hw_plan *const *plans, int n, int tile, int64_t steps,
                    hipStream_t s)
{
    hw_status st;
    bool direct = false;
    for (int i = 0; i < n; ++i)
        direct = direct || plans[i]->direct;
    const int per = group_steps(plans, n, tile);      // steps per launch
    const int64_t graph_launches = kGraphSteps / per;
    if (!direct && steps >= kGraphSteps + 1 && n == 1) {
        hw_plan *p = plans[0];
        if (p->cur != 0) {                 // align to the captured field set
            if ((st = launch_group(plans, 1, tile, s, true)) != HW_OK)
                return st;
            steps -= 1;
        }
        if (!p->graph || p->graph_tile != tile) {
            if (p->graph) {
                (void)hipGraphExecDestroy(p->graph);
                p->graph = nullptr;
            }
            if ((st = capture_stream(&p->cap_stream)) != HW_OK ||
                (st = capture_run(plans, 1, tile, p->cap_stream, &p->graph)) != HW_OK)
                return st;
            p->graph_tile = tile;
        }
        for (; steps >= kGraphSteps; steps -= kGraphSteps) {
            HW_HIP(hipGraphLaunch(p->graph, s));
            advance_state(plans, 1, kGraphSteps, graph_launches);
        }
    } else if (!direct && steps >= 2 * kGraphSteps) {
        hipGraphExec_t exec = nullptr;
        reap_graphs(false);
        if ((st = capture_stream(&t_cap_stream)) != HW_OK ||
            (st = capture_run(plans, n, tile, t_cap_stream, &exec)) != HW_OK)
            return st;
        for (; steps >= kGraphSteps; steps -= kGraphSteps) {
            hipError_t e = hipGraphLaunch(exec, s);
            if (e != hipSuccess) {
                (void)retire_graph(exec, s);
                return fail(HW_E_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
            }
            advance_state(plans, n, kGraphSteps, graph_launches);
        }
        if ((st = retire_graph(exec, s)) != HW_OK)
            return st;
    }
    for (; steps >= per; steps -= per)
        if ((st = launch_group(plans, n, tile, s)) != HW_OK)
            return st;
    for (; steps > 0; --steps)             // a last single step of a two-step shape
        if ((st = launch_group(plans, n, tile, s, true)) != HW_OK)
            return st;
    return HW_OK;
}

hw_status record_energy(hw_plan *p, hipStream_t s)
{
    if (p->trace_n >= p->pb.trace_cap)
        return fail(HW_E_NOMEM, "energy trace is full");
    hipError_t e;
    double factor = 0.5 * p->pb.dx * p->pb.dx * p->scale_down * p->scale_down;
    if (p->pb.physics == HW_ACOUSTIC2D) {
        e = launch_ac2d_energy((const Ac2dDesc *)p->d_desc, p->cur, p->pb.ny,
                               p->pb.storage, p->pb.order, p->L.words,
                               p->partial, s);
    } else if (p->pb.physics == HW_ELASTIC2D) {
        e = launch_el2d_energy((const El2dDesc *)p->d_desc, p->cur, p->pb.ny,
                               p->pb.storage, p->L.words, p->partial, s);
    } else {
        factor *= p->pb.dx;
        e = launch_el3d_energy((const El3dDesc *)p->d_desc, p->cur, p->L.rows,
                               p->pb.storage, p->L.words, p->partial, s);
    }
    if (e == hipSuccess)
        e = launch_energy_finish(p->partial, p->L.rows, factor,
                                 p->trace + p->trace_n, p->flags, s);
    if (e != hipSuccess)
        return fail(HW_E_DEVICE, std::string("energy launch: ") + hipGetErrorString(e));
    p->trace_steps.push_back(p->step);
    p->trace_n += 1;
    p->last_logged = p->step;
    return HW_OK;
}

int64_t logs_needed(const hw_plan *p, int64_t nsteps, int64_t every)
{
    if (every <= 0)
        return 0;
    int64_t first = p->step + (every - p->step % every) % every;   // >= step
    int64_t last = p->step + nsteps;
    if (first > last)
        return 0;
    int64_t cnt = (last - first) / every + 1;
    if (first == p->last_logged)
        cnt -= 1;
    return cnt;
}

hw_status check_ready(const hw_plan *p)
{
    if (!p)
        return fail(HW_E_INVAL, "plan is NULL");
    if (!p->have_material || !p->have_fields)
        return fail(HW_E_STATE, "material and fields must be uploaded first");
    return HW_OK;
}

hw_status host_fields_in_range(const hw_plan *p, const double *const *fields)
{
    if (p->pb.physics == HW_ELASTIC2D) {
        // syy vanishes on the free surfaces; vy and sxy have no row ny-1
        const int64_t nx = p->pb.nx, last = (p->pb.ny - 1) * nx;
        for (int64_t i = 0; i < nx; ++i)
            if ((fields[3] && (fields[3][i] != 0.0 || fields[3][last + i] != 0.0)) ||
                (fields[1] && fields[1][last + i] != 0.0) ||
                (fields[4] && fields[4][last + i] != 0.0))
                return fail(HW_E_INVAL, "elastic2d: syy must be zero on rows 0 and "
                                        "ny-1, vy and sxy zero on row ny-1");
    }
    const double maxv = max_finite(p->pb.storage);
    for (int f = 0; f < p->L.nf; ++f) {
        const double *a = fields[f];
        if (!a)
            continue;
        for (int64_t i = 0; i < p->L.cells; ++i) {
            const double v = a[i] * p->scale_up;
            if (!std::isfinite(v) || std::fabs(v) > maxv)
                return fail(HW_E_RANGE, "field " + std::to_string(f) + " value " +
                                            std::to_string(a[i]) + " at " +
                                            std::to_string(i) +
                                            " does not fit the storage format");
        }
    }
    return HW_OK;
}

hw_status host_material_ok(const hw_plan *p, const double *const *mat)
{
    const hw_problem &pb = p->pb;
    const int64_t nx = pb.nx, ny = pb.ny, nz = pb.nz, n = p->L.cells;
    const int nin = pb.physics == HW_ACOUSTIC2D ? 2 : 3;   // host arrays
    for (int m = 0; m < nin; ++m)
        if (!mat[m])
            return fail(HW_E_INVAL, "material array " + std::to_string(m) + " is NULL");
    for (int64_t i = 0; i < n; ++i) {
        const double rho = mat[0][i];
        if (!std::isfinite(rho) || !(rho > 0) || !std::isfinite((float)(1.0 / rho)) ||
            (float)(1.0 / rho) == 0.0f)
            return fail(HW_E_INVAL, "rho must be finite, > 0 and 1/rho must fit fp32");
        for (int m = 1; m < nin; ++m)
            if (!std::isfinite(mat[m][i]) || !std::isfinite((float)mat[m][i]))
                return fail(HW_E_INVAL, "material values must be finite in fp32");
        if (pb.physics == HW_ACOUSTIC2D) {
            if (!(mat[1][i] > 0))
                return fail(HW_E_INVAL, "kappa must be > 0");
        } else if (pb.physics == HW_ELASTIC2D) {
            // plane strain: positive shear and 2D bulk moduli (the plate
            // modulus of the surface rows is then positive as well)
            const double lam = mat[1][i], mu = mat[2][i];
            if (!(mu > 0) || !(lam + mu > 0))
                return fail(HW_E_INVAL, "need mu > 0 and lambda + mu > 0");
        } else {
            const double lam = mat[1][i], mu = mat[2][i];
            if (!(mu > 0) || !(3 * lam + 2 * mu > 0))
                return fail(HW_E_INVAL, "need mu > 0 and 3 lambda + 2 mu > 0");
        }
    }
    // Courant number: for every face, staggered buoyancy times the larger
    // modulus of the two cells it joins.
    double c2max = 0.0;
    auto idx = [&](int64_t i, int64_t j, int64_t k) {
        return ((k % nz) * ny + (j % ny)) * nx + (i % nx);
    };
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t q = idx(i, j, k);
                const int64_t nb[3] = {idx(i + 1, j, k), idx(i, j + 1, k), idx(i, j, k + 1)};
                const int naxes = pb.physics == HW_ELASTIC3D ? 3 : 2;
                for (int a = 0; a < naxes; ++a) {
                    const int64_t r = nb[a];
                    const double bf = 0.5 * (1.0 / mat[0][q] + 1.0 / mat[0][r]);
                    double mq, mr;
                    if (pb.physics == HW_ACOUSTIC2D) {
                        mq = mat[1][q];
                        mr = mat[1][r];
                    } else {
                        mq = mat[1][q] + 2 * mat[2][q];
                        mr = mat[1][r] + 2 * mat[2][r];
                    }
                    c2max = std::max(c2max, bf * std::max(mq, mr));
                }
            }
    const double cfl = std::sqrt(c2max) * pb.dt / pb.dx;
    const double bound = cfl_bound(pb.physics, pb.order);
    if (!(cfl < bound))
        return fail(HW_E_UNSTABLE, "Courant number " + std::to_string(cfl) +
                                       " is not below the stability bound " +
                                       std::to_string(bound));
    return HW_OK;
}

hw_status upload_desc(hw_plan *p, hipStream_t s)
{
    const int ph = p->pb.physics;
    const void *src = ph == HW_ACOUSTIC2D ? (const void *)&p->h2
                      : ph == HW_ELASTIC3D ? (const void *)&p->h3
                                           : (const void *)&p->he;
    const size_t n = ph == HW_ACOUSTIC2D ? sizeof(Ac2dDesc)
                     : ph == HW_ELASTIC3D ? sizeof(El3dDesc)
                                          : sizeof(El2dDesc);
    HW_HIP(hipMemcpyAsync(p->d_desc, src, n, hipMemcpyHostToDevice, s));
    return HW_OK;
}

hw_status advance_one(hw_plan *p, int64_t nsteps, int64_t every, hipStream_t s)
{
    hw_status st;
    if (every > 0 && p->step % every == 0 && p->last_logged != p->step)
        if ((st = record_energy(p, s)) != HW_OK)
            return st;
    hw_plan *pl[1] = {p};
    while (nsteps > 0) {
        int64_t chunk = nsteps;
        if (every > 0)
            chunk = std::min(chunk, every - p->step % every);
        if ((st = run_steps(pl, 1, p->tile, chunk, s)) != HW_OK)
            return st;
        nsteps -= chunk;
        if (every > 0 && p->step % every == 0)
            if ((st = record_energy(p, s)) != HW_OK)
                return st;
    }
    return HW_OK;
}

// Apply f to the descriptor that carries a 2D plan's source and receivers
// (the acoustic and the 2D elastic descriptors name them alike).
template <class F>
void on_forcing(hw_plan *p, F f)
{
    if (p->pb.physics == HW_ELASTIC2D)
        f(p->he);
    else
        f(p->h2);
}

// Point a plan's fields at the regions of its arena and fill its
// descriptors (host only).
void init_plan(hw_plan *p, const hw_problem *pb, const Layout &L, void *arena)
{
    p->pb = *pb;
    p->L = L;
    p->arena = (char *)arena;
    for (int s = 0; s < 2; ++s)
        for (int f = 0; f < 9; ++f) {
            const int ss = s < L.sets ? s : 0;
            p->fld[s][f] = f < L.nf ? p->arena + L.off_fld[ss][f] : nullptr;
        }
    for (int m = 0; m < 4; ++m)
        p->mat[m] = m < L.nm ? (float *)(p->arena + L.off_mat[m]) : nullptr;
    p->staging = (double *)(p->arena + L.off_staging);
    p->partial = (double *)(p->arena + L.off_partial);
    p->trace = (double *)(p->arena + L.off_trace);
    p->flags = (int32_t *)(p->arena + L.off_flags);
    p->d_desc = p->arena + L.off_desc;
    p->scale_up = std::ldexp(1.0, pb->scale_log2);
    p->scale_down = std::ldexp(1.0, -pb->scale_log2);
    const double r = pb->dt / pb->dx;
    if (pb->physics == HW_ACOUSTIC2D) {
        Ac2dDesc &d = p->h2;
        std::memset(&d, 0, sizeof(d));
        d.nx = pb->nx;
        d.ny = pb->ny;
        d.pitch = L.pitch;
        d.w1 = pb->order == 4 ? (float)((9.0 / 8.0) * r) : (float)(1.0 * r);
        d.w2 = pb->order == 4 ? (float)((-1.0 / 24.0) * r) : 0.0f;
        d.b = p->mat[0];
        d.k = p->mat[1];
        for (int s = 0; s < 2; ++s) {
            d.vx[s] = p->fld[s][0];
            d.vy[s] = p->fld[s][1];
            d.p[s] = p->fld[s][2];
        }
        d.comp_off = (int64_t)L.comp_off;
        p->counter = (int64_t *)(p->arena + L.off_flags + 8);
        d.step = p->counter;
        d.src = (const float *)(p->arena + L.off_src);
        d.rec_xy = (const int32_t *)(p->arena + L.off_recxy);
        d.rec = (double *)(p->arena + L.off_rec);
        d.rec_rows = pb->rec_steps;
        d.rec_scale = p->scale_down;
    } else if (pb->physics == HW_ELASTIC2D) {
        El2dDesc &d = p->he;
        std::memset(&d, 0, sizeof(d));
        d.nx = pb->nx;
        d.ny = pb->ny;
        d.pitch = L.pitch;
        d.w = (float)(1.0 * r);
        d.b = p->mat[0];
        d.l2m = p->mat[1];
        d.lam = p->mat[2];
        d.mxy = p->mat[3];
        for (int s = 0; s < 2; ++s)
            for (int f = 0; f < 5; ++f)
                d.f[s][f] = p->fld[s][f];
        p->counter = (int64_t *)(p->arena + L.off_flags + 8);
        d.step = p->counter;
        d.src = (const float *)(p->arena + L.off_src);
        d.rec_xy = (const int32_t *)(p->arena + L.off_recxy);
        d.rec = (double *)(p->arena + L.off_rec);
        d.rec_rows = pb->rec_steps;
        d.rec_scale = p->scale_down;
    } else {
        El3dDesc &d = p->h3;
        std::memset(&d, 0, sizeof(d));
        d.nx = pb->nx;
        d.ny = pb->ny;
        d.nz = pb->nz;
        d.pitch = L.pitch;
        d.slab = L.slab;
        d.w = (float)(1.0 * r);
        d.b = p->mat[0];
        d.lam = p->mat[1];
        d.mu = p->mat[2];
        for (int s = 0; s < 2; ++s)
            for (int f = 0; f < 9; ++f)
                d.f[s][f] = p->fld[s][f];
    }
}

// The body of hw_simulate on a plan: upload, advance, download.  Every
// region of the arena that a kernel reads before writing (both field sets,
// the status flags and the step counter) is cleared by hw_set_fields.
hw_status simulate_plan(hw_plan *p, const double *const *material, double *const *fields,
                        int64_t nsteps, int64_t energy_every, double *energy,
                        int64_t energy_cap, int64_t *n_energy, void *stream);

struct BlobHeader {
    char magic[8];
    uint32_t abi;
    int32_t physics, order, storage, comp, scale_log2;
    int64_t nx, ny, nz, step;
    uint64_t field_bytes;
};

}  // namespace

// ------------------------------------------------------------------ ABI --

extern "C" {

uint32_t hw_abi_version(void) { return HW_ABI_VERSION; }

const char *hw_last_error(void) { return g_error.c_str(); }

int32_t hw_num_fields(int32_t physics)
{
    return physics == HW_ACOUSTIC2D ? 3 : physics == HW_ELASTIC3D ? 9
                                        : physics == HW_ELASTIC2D ? 5 : 0;
}

int32_t hw_num_materials(int32_t physics)
{
    return physics == HW_ACOUSTIC2D ? 2
           : physics == HW_ELASTIC3D || physics == HW_ELASTIC2D ? 3 : 0;
}

double hw_cfl_bound(int32_t physics, int32_t order) { return cfl_bound(physics, order); }

hw_status hw_footprint(const hw_problem *pb, size_t *device_bytes)
{
    hw_status st = validate(pb);
    if (st != HW_OK)
        return st;
    if (!device_bytes)
        return fail(HW_E_INVAL, "device_bytes is NULL");
    *device_bytes = make_layout(pb).total;
    return HW_OK;
}

hw_status hw_plan_create(const hw_problem *pb, void *arena, size_t arena_bytes,
                         hw_plan **out)
{
    hw_status st = validate(pb);
    if (st != HW_OK)
        return st;
    if (!out)
        return fail(HW_E_INVAL, "out is NULL");
    if (!arena || ((uintptr_t)arena % kAlign) != 0)
        return fail(HW_E_INVAL, "arena must be a non-NULL 256-byte aligned device pointer");
    const Layout L = make_layout(pb);
    if (arena_bytes < L.total)
        return fail(HW_E_NOMEM, "arena has " + std::to_string(arena_bytes) +
                                    " bytes, the plan needs " + std::to_string(L.total));
    hw_plan *p = new (std::nothrow) hw_plan();
    if (!p)
        return fail(HW_E_NOMEM, "host allocation failed");
    init_plan(p, pb, L, arena);
    *out = p;
    return HW_OK;
}

void hw_plan_destroy(hw_plan *plan) { delete plan; }

hw_status hw_set_material(hw_plan *p, const double *const *material, void *stream)
{
    if (!p || !material)
        return fail(HW_E_INVAL, "plan or material is NULL");
    hw_status st = host_material_ok(p, material);
    if (st != HW_OK)
        return st;
    hipStream_t s = S(stream);
    const int64_t nx = p->pb.nx;
    if (p->pb.physics == HW_ELASTIC2D) {
        // The step's per-cell coefficients, each computed in fp64 and
        // rounded once to fp32 on the device: lambda + 2 mu and lambda, on
        // the two surface rows the plate modulus 4 mu (lambda + mu) /
        // (lambda + 2 mu) and 0 (syy = 0 eliminates the vertical strain
        // rate); and mu at each sxy point, the mean of the four cells
        // around it (rows 0 .. ny-2).
        const int64_t ny = p->pb.ny, n = p->L.cells;
        const double *lam = material[1], *mu = material[2];
        std::vector<double> tab[3];
        for (auto &t : tab)
            t.assign((size_t)n, 0.0);
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t q = j * nx + i, qx = j * nx + (i + 1) % nx;
                const bool surface = j == 0 || j == ny - 1;
                tab[0][q] = surface ? (4.0 * mu[q] * (lam[q] + mu[q])) / (lam[q] + 2.0 * mu[q])
                                    : lam[q] + 2.0 * mu[q];
                tab[1][q] = surface ? 0.0 : lam[q];
                if (j < ny - 1)
                    tab[2][q] = 0.25 * ((mu[q] + mu[qx]) + (mu[q + nx] + mu[qx + nx]));
            }
        for (int m = 0; m < p->L.nm; ++m) {
            const double *src = m == 0 ? material[0] : tab[m - 1].data();
            HW_HIP(hipMemcpyAsync(p->staging, src, (size_t)n * 8, hipMemcpyHostToDevice, s));
            HW_HIP(launch_material(p->staging, p->mat[m], m == 0, nx, p->L.rows,
                                   p->L.pitch, s));
        }
        if ((st = upload_desc(p, s)) != HW_OK)
            return st;
        HW_HIP(hipStreamSynchronize(s));     // the tables are local
        p->have_material = true;
        return HW_OK;
    }
    for (int m = 0; m < p->L.nm; ++m) {
        HW_HIP(hipMemcpyAsync(p->staging, material[m], (size_t)p->L.cells * 8,
                              hipMemcpyHostToDevice, s));
        HW_HIP(launch_material(p->staging, p->mat[m], m == 0, nx, p->L.rows,
                               p->L.pitch, s));
    }
    if ((st = upload_desc(p, s)) != HW_OK)
        return st;
    p->have_material = true;
    return HW_OK;
}

hw_status hw_set_fields(hw_plan *p, const double *const *fields, void *stream)
{
    if (!p || !fields)
        return fail(HW_E_INVAL, "plan or fields is NULL");
    hw_status st = host_fields_in_range(p, fields);
    if (st != HW_OK)
        return st;
    hipStream_t s = S(stream);
    for (int f = 0; f < p->L.nf; ++f) {
        // zero values and compensation terms, then write the values; the
        // other field set is cleared too, since the kernels never write its
        // padding and an exported state must not depend on the arena's past
        HW_HIP(launch_fill_zero(p->fld[0][f], p->L.field_bytes, s));
        if (p->L.sets > 1)
            HW_HIP(launch_fill_zero(p->fld[1][f], p->L.field_bytes, s));
        if (!fields[f])
            continue;
        HW_HIP(hipMemcpyAsync(p->staging, fields[f], (size_t)p->L.cells * 8,
                              hipMemcpyHostToDevice, s));
        HW_HIP(launch_to_storage(p->staging, p->fld[0][f], p->pb.storage, p->pb.nx,
                                 p->L.rows, p->L.pitch, p->L.words, 0,
                                 p->scale_up, s));
    }
    HW_HIP(launch_fill_zero(p->flags, kAlign, s));
    if ((st = upload_desc(p, s)) != HW_OK)
        return st;
    p->cur = 0;
    p->step = 0;
    p->trace_n = 0;
    p->last_logged = -1;
    p->trace_steps.clear();
    p->have_fields = true;
    return HW_OK;
}

hw_status hw_advance(hw_plan *p, int64_t nsteps, int64_t energy_every, void *stream)
{
    hw_status st = check_ready(p);
    if (st != HW_OK)
        return st;
    if (nsteps < 0)
        return fail(HW_E_INVAL, "nsteps must be >= 0");
    if (p->trace_n + logs_needed(p, nsteps, energy_every) > p->pb.trace_cap)
        return fail(HW_E_NOMEM, "energy trace capacity too small for this advance");
    return advance_one(p, nsteps, energy_every, S(stream));
}

hw_status hw_record_energy(hw_plan *p, void *stream)
{
    hw_status st = check_ready(p);
    if (st != HW_OK)
        return st;
    return record_energy(p, S(stream));
}

hw_status hw_energy_trace(hw_plan *p, double *energy, int64_t *step, int64_t cap,
                          int64_t *n_out, void *stream)
{
    if (!p)
        return fail(HW_E_INVAL, "plan is NULL");
    hipStream_t s = S(stream);
    std::vector<double> e((size_t)std::max<int64_t>(p->trace_n, 1));
    int32_t flag = 0;
    if (p->trace_n > 0)
        HW_HIP(hipMemcpyAsync(e.data(), p->trace, (size_t)p->trace_n * 8,
                              hipMemcpyDeviceToHost, s));
    HW_HIP(hipMemcpyAsync(&flag, p->flags, 4, hipMemcpyDeviceToHost, s));
    HW_HIP(hipStreamSynchronize(s));
    const int64_t n = std::min(cap, p->trace_n);
    for (int64_t k = 0; k < n; ++k) {
        if (energy)
            energy[k] = e[k];
        if (step)
            step[k] = p->trace_steps[k];
    }
    if (n_out)
        *n_out = p->trace_n;
    if (flag)
        return fail(HW_E_NONFINITE, "the state became non-finite");
    return HW_OK;
}

hw_status hw_get_fields(hw_plan *p, double *const *fields, double *const *comps,
                        void *stream)
{
    hw_status st = check_ready(p);
    if (st != HW_OK)
        return st;
    hipStream_t s = S(stream);
    const size_t bytes = (size_t)p->L.cells * 8;
    for (int pass = 0; pass < 2; ++pass) {
        double *const *dst = pass == 0 ? fields : comps;
        if (!dst)
            continue;
        for (int f = 0; f < p->L.nf; ++f) {
            if (!dst[f])
                continue;
            if (pass == 1 && p->pb.comp == HW_COMP_NONE) {
                std::memset(dst[f], 0, bytes);
                continue;
            }
            if (pass == 1 && p->L.c8)
                HW_HIP(launch_comp8_to_double(p->fld[p->cur][f], p->L.comp_off,
                                              p->staging, p->pb.storage, p->pb.nx,
                                              p->L.rows, p->L.pitch, p->scale_down, s));
            else
                HW_HIP(launch_from_storage(p->fld[p->cur][f], p->staging, p->pb.storage,
                                           p->pb.nx, p->L.rows, p->L.pitch, p->L.words,
                                           pass, p->scale_down, s));
            HW_HIP(hipMemcpyAsync(dst[f], p->staging, bytes, hipMemcpyDeviceToHost, s));
        }
    }
    int32_t flag = 0;
    HW_HIP(hipMemcpyAsync(&flag, p->flags, 4, hipMemcpyDeviceToHost, s));
    HW_HIP(hipStreamSynchronize(s));
    if (flag)
        return fail(HW_E_NONFINITE, "the state became non-finite");
    return HW_OK;
}

int64_t hw_plan_step(const hw_plan *p) { return p ? p->step : -1; }

hw_status hw_state_size(const hw_plan *p, size_t *bytes)
{
    if (!p || !bytes)
        return fail(HW_E_INVAL, "plan or bytes is NULL");
    *bytes = sizeof(BlobHeader) + (size_t)p->L.nf * p->L.field_bytes;
    return HW_OK;
}

hw_status hw_state_export(hw_plan *p, void *blob, size_t bytes, void *stream)
{
    hw_status st = check_ready(p);
    if (st != HW_OK)
        return st;
    size_t need;
    hw_state_size(p, &need);
    if (!blob || bytes < need)
        return fail(HW_E_INVAL, "blob too small");
    BlobHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, "HWSTATE1", 8);
    h.abi = HW_ABI_VERSION;
    h.physics = p->pb.physics;
    h.order = p->pb.order;
    h.storage = p->pb.storage;
    h.comp = p->pb.comp;
    h.scale_log2 = p->pb.scale_log2;
    h.nx = p->pb.nx;
    h.ny = p->pb.ny;
    h.nz = p->pb.nz;
    h.step = p->step;
    h.field_bytes = p->L.field_bytes;
    std::memcpy(blob, &h, sizeof(h));
    char *dst = (char *)blob + sizeof(h);
    hipStream_t s = S(stream);
    for (int f = 0; f < p->L.nf; ++f, dst += p->L.field_bytes)
        HW_HIP(hipMemcpyAsync(dst, p->fld[p->cur][f], p->L.field_bytes,
                              hipMemcpyDeviceToHost, s));
    HW_HIP(hipStreamSynchronize(s));
    return HW_OK;
}

hw_status hw_state_import(hw_plan *p, const void *blob, size_t bytes, void *stream)
{
    if (!p || !blob)
        return fail(HW_E_INVAL, "plan or blob is NULL");
    if (!p->have_material)
        return fail(HW_E_STATE, "upload the material before importing a state");
    size_t need;
    hw_state_size(p, &need);
    if (bytes < need)
        return fail(HW_E_INVAL, "blob too small");
    BlobHeader h;
    std::memcpy(&h, blob, sizeof(h));
    if (std::memcmp(h.magic, "HWSTATE1", 8) != 0 || h.abi != HW_ABI_VERSION ||
        h.physics != p->pb.physics || h.order != p->pb.order ||
        h.storage != p->pb.storage || h.comp != p->pb.comp ||
        h.scale_log2 != p->pb.scale_log2 || h.nx != p->pb.nx ||
        h.ny != p->pb.ny || h.nz != p->pb.nz ||
        h.field_bytes != p->L.field_bytes || h.step < 0)
        return fail(HW_E_INVAL, "blob does not match this plan's problem");
    hipStream_t s = S(stream);
    const char *src = (const char *)blob + sizeof(h);
    for (int f = 0; f < p->L.nf; ++f, src += p->L.field_bytes) {
        HW_HIP(hipMemcpyAsync(p->fld[0][f], src, p->L.field_bytes,
                              hipMemcpyHostToDevice, s));
        if (p->L.sets > 1)         // padding of the other set (see hw_set_fields)
            HW_HIP(launch_fill_zero(p->fld[1][f], p->L.field_bytes, s));
    }
    HW_HIP(launch_fill_zero(p->flags, kAlign, s));
    if (p->counter)
        HW_HIP(launch_set_counter(p->counter, h.step, s));
    HW_HIP(hipStreamSynchronize(s));
    p->cur = 0;
    p->step = h.step;
    p->trace_n = 0;
    p->last_logged = -1;
    p->trace_steps.clear();
    p->have_fields = true;
    return HW_OK;
}

hw_status hw_set_source(hw_plan *p, int64_t ix, int64_t iy, const double *samples,
                        int64_t nsamples, void *stream)
{
    if (!p)
        return fail(HW_E_INVAL, "plan is NULL");
    if (p->pb.physics == HW_ELASTIC3D)
        return fail(HW_E_INVAL, "sources are 2D only");
    if (nsamples < 0 || (nsamples > 0 && !samples))
        return fail(HW_E_INVAL, "bad sample array");
    if (nsamples > p->pb.src_cap)
        return fail(HW_E_NOMEM, "more samples than src_cap");
    if (nsamples > 0 && (ix < 0 || ix >= p->pb.nx || iy < 0 || iy >= p->pb.ny))
        return fail(HW_E_INVAL, "source cell outside the grid");
    if (nsamples > 0 && p->pb.physics == HW_ELASTIC2D && iy > p->pb.ny - 2)
        return fail(HW_E_INVAL, "elastic2d: the vy source row must be <= ny-2");
    std::vector<float> v((size_t)nsamples);
    for (int64_t n = 0; n < nsamples; ++n) {
        if (!std::isfinite(samples[n]) || !std::isfinite((float)samples[n]))
            return fail(HW_E_RANGE, "source sample not finite in fp32");
        v[(size_t)n] = (float)samples[n];     // round to nearest even
    }
    hipStream_t s = S(stream);
    HW_HIP(hipStreamSynchronize(s));
    const float *dsrc = nullptr;
    on_forcing(p, [&](auto &d) { dsrc = d.src; });
    if (nsamples > 0)
        HW_HIP(hipMemcpy((void *)dsrc, v.data(), v.size() * 4, hipMemcpyHostToDevice));
    on_forcing(p, [&](auto &d) {
        d.src_n = nsamples;
        d.src_x = (int32_t)(nsamples > 0 ? ix : 0);
        d.src_y = (int32_t)(nsamples > 0 ? iy : 0);
    });
    hw_status st = upload_desc(p, s);
    if (st == HW_OK && p->graph) {      // the captured launches hold the old descriptor
        (void)hipGraphExecDestroy(p->graph);
        p->graph = nullptr;
    }
    if (st == HW_OK)
        HW_HIP(hipStreamSynchronize(s));
    return st;
}

hw_status hw_set_receivers(hw_plan *p, int32_t n, const int64_t *ix, const int64_t *iy,
                           void *stream)
{
    if (!p)
        return fail(HW_E_INVAL, "plan is NULL");
    if (p->pb.physics == HW_ELASTIC3D)
        return fail(HW_E_INVAL, "receivers are 2D only");
    if (n < 0 || (n > 0 && (!ix || !iy)))
        return fail(HW_E_INVAL, "bad receiver arrays");
    if (n > p->pb.rec_cap)
        return fail(HW_E_NOMEM, "more receivers than rec_cap");
    std::vector<int32_t> xy((size_t)n * 2);
    for (int32_t r = 0; r < n; ++r) {
        if (ix[r] < 0 || ix[r] >= p->pb.nx || iy[r] < 0 || iy[r] >= p->pb.ny)
            return fail(HW_E_INVAL, "receiver cell outside the grid");
        xy[2 * (size_t)r] = (int32_t)ix[r];
        xy[2 * (size_t)r + 1] = (int32_t)iy[r];
    }
    hipStream_t s = S(stream);
    HW_HIP(hipStreamSynchronize(s));
    const int32_t *dxy = nullptr;
    on_forcing(p, [&](auto &d) { dxy = d.rec_xy; });
    if (n > 0)
        HW_HIP(hipMemcpy((void *)dxy, xy.data(), xy.size() * 4, hipMemcpyHostToDevice));
    on_forcing(p, [&](auto &d) { d.rec_n = n; });
    hw_status st = upload_desc(p, s);
    if (st == HW_OK && p->graph) {
        (void)hipGraphExecDestroy(p->graph);
        p->graph = nullptr;
    }
    if (st == HW_OK)
        HW_HIP(hipStreamSynchronize(s));
    return st;
}

hw_status hw_receiver_trace(hw_plan *p, double *out, int64_t cap_rows, int64_t *rows_out,
                            void *stream)
{
    if (!p)
        return fail(HW_E_INVAL, "plan is NULL");
    if (p->pb.physics == HW_ELASTIC3D)
        return fail(HW_E_INVAL, "receivers are 2D only");
    const int64_t rows = std::min(p->step, p->pb.rec_steps);
    if (rows_out)
        *rows_out = rows;
    hipStream_t s = S(stream);
    const int64_t k = std::min(rows, std::max<int64_t>(cap_rows, 0));
    int32_t rn = 0;
    const double *rec = nullptr;
    on_forcing(p, [&](auto &d) {
        rn = d.rec_n;
        rec = d.rec;
    });
    if (out && k > 0 && rn > 0)
        HW_HIP(hipMemcpyAsync(out, rec, (size_t)k * rn * p->L.rec_vals * 8,
                              hipMemcpyDeviceToHost, s));
    HW_HIP(hipStreamSynchronize(s));
    return HW_OK;
}

int32_t hw_tile_count(int32_t physics)
{
    return tile_count(physics);
}

hw_status hw_tile_info(int32_t physics, int32_t tile, int32_t *tx, int32_t *ty,
                       int32_t *tz, int32_t *kind)
{
    if (tile < 0 || tile >= hw_tile_count(physics))
        return fail(HW_E_INVAL, "tile index out of range");
    const TileShape t = tile_table(physics)[tile];
    if (tx)
        *tx = t.tx;
    if (ty)
        *ty = t.ty;
    if (tz)
        *tz = t.tz;
    if (kind)
        *kind = t.kind;
    return HW_OK;
}

hw_status hw_plan_set_tile(hw_plan *p, int32_t tile)
{
    if (!p)
        return fail(HW_E_INVAL, "plan is NULL");
    if (tile < 0 || tile >= num_tiles(p->pb))
        return fail(HW_E_INVAL, "tile index out of range");
    if (p->pb.physics == HW_ACOUSTIC2D && p->pb.comp == HW_COMP_TWOSUM8 &&
        kTiles2D[tile].kind == 1)
        return fail(HW_E_INVAL, "8-bit compensation words do not run on the marching "
                                "kind 1");
    p->tile = tile;
    return HW_OK;
}

hw_status hw_batch_advance(hw_plan *const *plans, int32_t n, const int64_t *nsteps,
                           int64_t energy_every, int32_t tile, void *stream)
{
    if (!plans || !nsteps || n <= 0)
        return fail(HW_E_INVAL, "need n > 0 plans and their step counts");
    for (int i = 0; i < n; ++i) {
        hw_status st = check_ready(plans[i]);
        if (st != HW_OK)
            return st;
        if (nsteps[i] < 0)
            return fail(HW_E_INVAL, "nsteps must be >= 0");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i])
                return fail(HW_E_INVAL, "plans must be distinct");
        if (plans[i]->trace_n + logs_needed(plans[i], nsteps[i], energy_every) >
            plans[i]->pb.trace_cap)
            return fail(HW_E_NOMEM, "energy trace capacity too small for plan " +
                                        std::to_string(i));
        if (tile >= num_tiles(plans[i]->pb))
            return fail(HW_E_INVAL, "tile index out of range");
    }
    hipStream_t s = S(stream);
    hw_status st;
    std::vector<int64_t> left(nsteps, nsteps + n);
    for (int i = 0; i < n; ++i) {
        hw_plan *p = plans[i];
        if (energy_every > 0 && p->step % energy_every == 0 && p->last_logged != p->step)
            if ((st = record_energy(p, s)) != HW_OK)
                return st;
    }
    for (;;) {
        // the active set and every plan's next energy log fix the chunk
        std::map<KernelKey, std::vector<hw_plan *>> groups;
        std::vector<int> active;
        int64_t chunk = INT64_MAX;
        for (int i = 0; i < n; ++i)
            if (left[i] > 0) {
                groups[plans[i]->key()].push_back(plans[i]);
                active.push_back(i);
                chunk = std::min(chunk, left[i]);
                if (energy_every > 0)
                    chunk = std::min(chunk, energy_every - plans[i]->step % energy_every);
            }
        if (active.empty())
            break;
        for (auto &g : groups) {
            const int t = tile >= 0 ? tile : g.second[0]->tile;
            if ((st = run_steps(g.second.data(), (int)g.second.size(), t, chunk, s)) != HW_OK)
                return st;
        }
        for (int i : active) {
            left[i] -= chunk;
            hw_plan *p = plans[i];
            if (energy_every > 0 && p->step % energy_every == 0)
                if ((st = record_energy(p, s)) != HW_OK)
                    return st;
        }
    }
    return HW_OK;
}

hw_status hw_simulate(const hw_problem *pb, const double *const *material,
                      double *const *fields, int64_t nsteps, int64_t energy_every,
                      double *energy, int64_t energy_cap, int64_t *n_energy,
                      void *arena, size_t arena_bytes, void *stream)
{
    if (!fields)
        return fail(HW_E_INVAL, "fields is NULL");
    hw_plan *p = nullptr;
    hw_status st = hw_plan_create(pb, arena, arena_bytes, &p);
    if (st != HW_OK)
        return st;
    st = simulate_plan(p, material, fields, nsteps, energy_every, energy, energy_cap,
                       n_energy, stream);
    hw_plan_destroy(p);
    return st;
}

hw_status hw_simulate_noalloc(const hw_problem *pb, const double *const *material,
                              double *const *fields, int64_t nsteps,
                              int64_t energy_every, double *energy,
                              int64_t energy_cap, int64_t *n_energy, void *stream)
{
    if (!fields)
        return fail(HW_E_INVAL, "fields is NULL");
    hw_status st = validate(pb);
    if (st != HW_OK)
        return st;
    const Layout L = make_layout(pb);
    if (L.total > (size_t)HW_NOALLOC_MAX_BYTES)
        return fail(HW_E_NOMEM, "problem needs " + std::to_string(L.total) +
                                    " device bytes; hw_simulate_noalloc holds at most " +
                                    std::to_string((size_t)HW_NOALLOC_MAX_BYTES));
    void *base = nullptr;
    if ((st = scratch_address(&base)) != HW_OK)
        return st;
    hw_plan p;                     // host object on the stack, arena = scratch
    init_plan(&p, pb, L, base);
    p.direct = true;
    st = simulate_plan(&p, material, fields, nsteps, energy_every, energy, energy_cap,
                       n_energy, stream);
    if (st != HW_OK)               // leave nothing in flight on the shared array
        (void)hipStreamSynchronize(S(stream));
    return st;
}

}  // extern "C"

namespace {

// The shape hw_simulate and hw_simulate_noalloc run: the one the tuning
// measurements pick at most sizes -- 2D acoustic: two steps per launch on
// 64 x 24 tiles; 3D elastic: the fused pass on 64 x 6 columns of 128
// planes -- and shape 0 for 2D elastic.  Every shape gives the same bits.
int simulate_tile(int physics)
{
    if (physics == HW_ACOUSTIC2D)
        for (int t = 0; t < kNumTiles2D; ++t)
            if (kTiles2D[t].kind == 5 && kTiles2D[t].ty == 24)
                return t;
    if (physics == HW_ELASTIC3D)
        for (int t = 0; t < kNumTiles3D; ++t)
            if (kTiles3D[t].kind == 2 && kTiles3D[t].ty == 6 && kTiles3D[t].tz == 128)
                return t;
    return 0;
}

hw_status simulate_plan(hw_plan *p, const double *const *material, double *const *fields,
                        int64_t nsteps, int64_t energy_every, double *energy,
                        int64_t energy_cap, int64_t *n_energy, void *stream)
{
    const double *const *in = (const double *const *)fields;
    hw_status st = hw_plan_set_tile(p, simulate_tile(p->pb.physics));
    if (st == HW_OK &&
        (st = hw_set_material(p, material, stream)) == HW_OK &&
        (st = hw_set_fields(p, in, stream)) == HW_OK &&
        (st = hw_advance(p, nsteps, energy_every, stream)) == HW_OK &&
        (st = hw_get_fields(p, fields, nullptr, stream)) == HW_OK)
        st = hw_energy_trace(p, energy, nullptr, energy_cap, n_energy, stream);
    return st;
}

}  // namespace
