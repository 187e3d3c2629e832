// Host side of libglbm: contexts, the C ABI of include/glbm.h, chunked stepping
// with HIP graph replay, checks and timing.
#include "glbm.h"
#include "glbm_cnn.h"
#include "glbm_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

using namespace glbm;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(GLBM_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                                \
    } while (0)

size_t store_bytes(int store)
{
    return store == GLBM_STORE_F64 ? 8 : ((store == GLBM_STORE_F32 || store == GLBM_STORE_F32LOC) ? 4 : 2);
}
// planes per instance and buffer: q populations, plus a float density plane
// (two half-width planes) for F16LOC
int planes_of(const glbm_instance_desc& d)
{
    return d.lattice + (d.store == GLBM_STORE_F16LOC ? 2 : (d.store == GLBM_STORE_F32LOC ? 1 : 0));
}
size_t compute_bytes(int store) { return store == GLBM_STORE_F64 ? 8 : 4; }
int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Plane stride: a multiple of 128 elements plus 128, so that the q planes of a
// power-of-two grid do not all start at the same offset modulo large powers
// of two (HBM channel interleave).
int64_t plane_stride(int64_t n) { return round_up(n, 128) + 128; }

int validate(int32_t n_inst, const glbm_instance_desc* d)
{
    if (n_inst < 1 || !d) return fail(GLBM_EINVAL, "n_inst must be >= 1");
    for (int i = 0; i < n_inst; ++i) {
        const glbm_instance_desc& x = d[i];
        if (x.lattice != GLBM_D2Q9 && x.lattice != GLBM_D3Q19)
            return fail(GLBM_EINVAL, "instance %d: lattice must be 9 or 19", i);
        if (x.store < 0 || x.store > 4) return fail(GLBM_EINVAL, "instance %d: bad store %d", i, x.store);
        if (x.nx < 1 || x.ny < 1 || x.nz < 1) return fail(GLBM_EINVAL, "instance %d: empty grid", i);
        if (x.lattice == GLBM_D2Q9 && x.nz != 1) return fail(GLBM_EINVAL, "instance %d: D2Q9 needs nz = 1", i);
        if (round_up((int64_t)x.nx * x.ny * x.nz, kBlk) * (x.lattice + 3) >= (int64_t)1 << 31)
            return fail(GLBM_EINVAL, "instance %d: grid too large for 32-bit plane indexing", i);
        if (!(x.tau > 0.5) || !std::isfinite(x.tau)) return fail(GLBM_EINVAL, "instance %d: tau must be > 1/2", i);
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(x.g[a])) return fail(GLBM_EINVAL, "instance %d: non-finite body force", i);
        if (x.check_every < 2 || (x.check_every & 1))
            return fail(GLBM_EINVAL, "instance %d: check_every must be even and >= 2", i);
        if (x.wall_faces & ~0x3Fu) return fail(GLBM_EINVAL, "instance %d: unknown wall face bits", i);
        for (int a = 0; a < 3; ++a)
            if (((x.wall_faces >> (2 * a)) & 1u) != ((x.wall_faces >> (2 * a + 1)) & 1u))
                return fail(GLBM_EINVAL, "instance %d: wall faces must come in pairs per axis", i);
        if ((x.store == GLBM_STORE_F16DEV || x.store == GLBM_STORE_F16LOC) && x.dev_scale_log2 != GLBM_SCALE_AUTO &&
            (x.dev_scale_log2 < 0 || x.dev_scale_log2 > 30))
            return fail(GLBM_EINVAL, "instance %d: dev_scale_log2 must be in [0, 30]", i);
        if (x.flags & ~(uint32_t)GLBM_FLAG_F16DEV_OPT_IN) return fail(GLBM_EINVAL, "instance %d: unknown flag bits", i);
        if (x.store == GLBM_STORE_F16DEV && !(x.flags & GLBM_FLAG_F16DEV_OPT_IN))
            return fail(GLBM_EINVAL,
                        "instance %d: GLBM_STORE_F16DEV resolves the velocity part of f only relative to the density "
                        "deviation (k several percent off on shale maps); use GLBM_STORE_F16LOC, or set "
                        "GLBM_FLAG_F16DEV_OPT_IN to run it as a study form",
                        i);
        if (x.lattice != d[0].lattice || x.store != d[0].store || x.check_every != d[0].check_every)
            return fail(GLBM_EINVAL, "instance %d: lattice, store and check_every must match instance 0", i);
        if (x.pressure_axis < 0 || x.pressure_axis > (x.lattice == GLBM_D2Q9 ? 2 : 3))
            return fail(GLBM_EINVAL, "instance %d: pressure_axis must be 0 (none) or 1 .. %d", i,
                        x.lattice == GLBM_D2Q9 ? 2 : 3);
        if ((x.pressure_axis != 0) != (d[0].pressure_axis != 0))
            return fail(GLBM_EINVAL, "instance %d: every instance of a context has pressure faces or none does", i);
        if (x.pressure_axis) {
            const int32_t na = x.pressure_axis == 1 ? x.nx : (x.pressure_axis == 2 ? x.ny : x.nz);
            if (na < 2) return fail(GLBM_EINVAL, "instance %d: the pressure axis needs at least 2 nodes", i);
            if (x.wall_faces)
                return fail(GLBM_EINVAL, "instance %d: pressure faces need periodic faces elsewhere (wall nodes are allowed)", i);
            if (!(x.rho_in > 0.0) || !(x.rho_out > 0.0) || !std::isfinite(x.rho_in) || !std::isfinite(x.rho_out) ||
                x.rho_in == x.rho_out)
                return fail(GLBM_EINVAL, "instance %d: face densities must be finite, > 0 and different", i);
        }
    }
    return GLBM_OK;
}

// Element layout of one population buffer.
struct Layout {
    std::vector<int64_t> off, stride;
    int64_t elems = 0;
};

Layout layout_of(int32_t n_inst, const glbm_instance_desc* d)
{
    Layout L;
    for (int i = 0; i < n_inst; ++i) {
        const int64_t n = (int64_t)d[i].nx * d[i].ny * d[i].nz;
        const int64_t s = plane_stride(node_blocks(d[i].store) ? round_up(n, kBlk) : n);
        L.off.push_back(L.elems);
        L.stride.push_back(s);
        L.elems += round_up(s * planes_of(d[i]), 256);
    }
    return L;
}

int auto_scale(const glbm_instance_desc& d)
{
    // F16DEV: deviations |f_i - w_i| of a slow body-force-driven flow stay far
    // below 2^-5; 2^20 keeps everything above 2^-34 in the normal FP16 range.
    // F16LOC: the stored part (velocity and non-equilibrium) is smaller still;
    // 2^24 covers 4e-12 .. 4e-3.
    return d.store == GLBM_STORE_F16LOC ? 24 : 20;
}

}  // namespace

void glbm::set_error(const char* msg) { g_err = msg; }

// ------------------------------------------------ allocation-free scratch --
// Staging of glbm_cnn_apply_noalloc (rho - 1 and three velocity planes of one
// instance, floats).  Each GPU holds its own copy until the process ends.  In
// host code the name `scratch` is only a stand-in for the symbol: kernels get
// the device address that hipGetSymbolAddress returns for the current device,
// fetched once per device when a context is created there.
static __device__ __align__(256) float scratch[4 * (size_t)GLBM_NOALLOC_MAX_NODES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (current at the call); GLBM_OK or GLBM_EDEVICE.
int fetch_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(GLBM_EDEVICE, "device %d outside the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return GLBM_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(GLBM_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
    return GLBM_OK;
}

float* scratch_of(int dev)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (dev >= 0 && dev < kMaxDevices) ? static_cast<float*>(g_scratch_ptr[dev]) : nullptr;
}
}  // namespace

struct glbm_ctx_s {
    int n_inst = 0;
    int device = 0;   // HIP device current at glbm_init_geometry
    Config cfg{};
    int n_c = 100;
    size_t esz = 0, tsz = 0;
    hipStream_t user = nullptr, work = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::vector<glbm_instance_desc> desc;
    std::vector<InstDev> inst_h;
    std::vector<Tile> tiles_h;
    std::vector<int64_t> n_fluid, steps, snap_step;
    std::vector<int32_t> active_h, dsteps_h, has_table;
    std::vector<std::vector<uint8_t>> cls_h;
    std::vector<std::vector<double>> eps_h, k_h;  // per-instance class tables as given
    int64_t gstep = 0;
    bool snap_valid = false;
    // device memory
    void* buf[2] = {nullptr, nullptr};
    bool own_pop = false;
    void* pop_base = nullptr;
    size_t pop_bytes = 0;
    uint8_t* cls_d = nullptr;
    InstDev* inst_d = nullptr;
    Tile* tiles_d = nullptr;
    void* tab_d = nullptr;
    void* snap_d = nullptr;
    double* part_d = nullptr;
    double* res_d = nullptr;
    double* flux_d = nullptr;
    int32_t* active_d = nullptr;
    int32_t* dsteps_d = nullptr;
    int64_t snap_elems = 0;
    // pinned host mirrors
    double* res_p = nullptr;
    int32_t* active_p = nullptr;
    // tiling and graph
    int tw_log2 = 6;   // tile width 2^tw_log2
    int th = 4;        // tile height
    int cache = 13;    // memory policy, see Args::cache (nontemporal stores, plain order, L1 table)
    bool staged_ok = false;  // D2Q9 FP16 store, periodic, every nx a multiple of 8: k_sweep9h applies
    bool paired_ok = false;  // D2Q9 FP16 store, periodic, every nx even: k_sweep9p applies
    int ntiles = 0;
    bool use_graph = true;
    hipGraphExec_t graph = nullptr;
    double graph_tol = 0.0;
    bool graph_valid = false;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_steps;  // sweeps covered by each recorded event pair
    size_t ev_used = 0;
    double time_ms = 0.0;
    int64_t launches = 0;

    // two steps per launch (cache policy bit 6): runs of 4k steps that start at
    // an even global step go as 2k two-step launches (an even count, so the state
    // ends in the buffer of its step parity), the rest as single steps
    bool tb_on() const { return (cache & 64) && tb_applies(cfg, tw_log2, th); }

    Args args(int parity) const
    {
        Args a{};
        a.tiles = tiles_d;
        a.inst = inst_d;
        a.cls = cls_d;
        a.buf[0] = buf[0];
        a.buf[1] = buf[1];
        a.tab = tab_d;
        a.snap = snap_d;
        a.part = part_d;
        a.res = res_d;
        a.active = active_d;
        a.dsteps = dsteps_d;
        a.ntiles = ntiles;
        a.parity = parity & 1;
        a.tw_log2 = tw_log2;
        a.nslot = ((1 << tw_log2) * th) / kBlock;
        a.cache = cache;
        a.staged = (staged_ok && (cache & 16) && tw_log2 <= 8 && (th == 1 || th == 2 || th == 4)) ? 1 : 0;
        a.paired = (paired_ok && !a.staged && (cache & 32) && tw_log2 >= 7 && a.nslot % 2 == 0) ? 1 : 0;
        return a;
    }
};

namespace {

void free_graph(glbm_ctx c)
{
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
    c->graph_valid = false;
}

int build_tiles(glbm_ctx c)
{
    c->tiles_h.clear();
    const int th = c->th, tw = 1 << c->tw_log2;
    for (int i = 0; i < c->n_inst; ++i) {
        InstDev& I = c->inst_h[i];
        I.tile0 = (int32_t)c->tiles_h.size();
        for (int z = 0; z < I.nz; ++z)
            for (int y = 0; y < I.ny; y += th)
                for (int x = 0; x < I.nx; x += tw) c->tiles_h.push_back(Tile{i, x, y, z});
        I.ntiles = (int32_t)c->tiles_h.size() - I.tile0;
    }
    c->ntiles = (int)c->tiles_h.size();
    if (c->tiles_d) (void)hipFree(c->tiles_d);
    if (c->part_d) (void)hipFree(c->part_d);
    c->tiles_d = nullptr;
    c->part_d = nullptr;
    HIPCHK(hipMalloc(&c->tiles_d, c->tiles_h.size() * sizeof(Tile)));
    HIPCHK(hipMalloc(&c->part_d, c->tiles_h.size() * kPartW * sizeof(double)));
    HIPCHK(hipMemcpyAsync(c->tiles_d, c->tiles_h.data(), c->tiles_h.size() * sizeof(Tile), hipMemcpyHostToDevice,
                          c->work));
    HIPCHK(hipMemcpyAsync(c->inst_d, c->inst_h.data(), c->inst_h.size() * sizeof(InstDev), hipMemcpyHostToDevice,
                          c->work));
    HIPCHK(hipStreamSynchronize(c->work));
    free_graph(c);
    return GLBM_OK;
}

// Default tile: one node per thread, 256 nodes along x (fewer if the grid is
// narrower), so each wavefront reads 64 consecutive nodes per plane and the
// lines straddled by x-shifted reads are shared by the four wavefronts.
void default_tile(glbm_ctx c)
{
    int max_nx = 1;
    for (auto& I : c->inst_h) max_nx = std::max(max_nx, I.nx);
    int twl = 6;
    while (twl < 8 && (1 << (twl + 1)) <= max_nx) ++twl;
    c->tw_log2 = twl;
    c->th = kBlock >> twl;
}

bool tile_ok(int tw_log2, int th)
{
    return tw_log2 >= 6 && tw_log2 <= 10 && th >= 1 && th <= 256 && (((1 << tw_log2) * th) % kBlock) == 0;
}

// Fork the work stream from the caller's stream.
int enter(glbm_ctx c)
{
    HIPCHK(hipEventRecord(c->ev_fork, c->user));
    HIPCHK(hipStreamWaitEvent(c->work, c->ev_fork, 0));
    return GLBM_OK;
}

// Join: make the caller's stream wait for the work queued so far.
int leave(glbm_ctx c)
{
    HIPCHK(hipEventRecord(c->ev_join, c->work));
    HIPCHK(hipStreamWaitEvent(c->user, c->ev_join, 0));
    return GLBM_OK;
}

// Joins the work stream back into the caller's stream on every exit path of an
// entry point that forked it, error returns included; done() joins explicitly
// and reports the join's own error.
struct Joined {
    glbm_ctx c;
    bool on = true;
    explicit Joined(glbm_ctx ctx) : c(ctx) {}
    Joined(const Joined&) = delete;
    Joined& operator=(const Joined&) = delete;
    ~Joined()
    {
        if (on) (void)leave(c);
    }
    int done()
    {
        on = false;
        return leave(c);
    }
};

int resolve_timing(glbm_ctx c)
{
    if (!c->ev_used) return GLBM_OK;
    HIPCHK(hipEventSynchronize(c->ev_pool[c->ev_used - 1]));
    for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->ev_pool[k], c->ev_pool[k + 1]));
        c->time_ms += ms;
        c->launches += c->ev_steps[k / 2];
    }
    c->ev_used = 0;
    c->ev_steps.clear();
    return GLBM_OK;
}

// One sweep, or with two = true one two-step launch (the caller keeps such
// launches in pairs within a chunk, so the state returns to the buffer of its
// step parity).
int sweep_once(glbm_ctx c, int parity, bool two = false)
{
    if (c->timing) {
        if (c->ev_used + 2 > c->ev_pool.size()) {
            int rc = resolve_timing(c);
            if (rc) return rc;
            while (c->ev_pool.size() < 512) {
                hipEvent_t e;
                HIPCHK(hipEventCreate(&e));
                c->ev_pool.push_back(e);
            }
        }
        HIPCHK(hipEventRecord(c->ev_pool[c->ev_used++], c->work));
        c->ev_steps.push_back(two ? 2 : 1);
    }
    if (two) HIPCHK(launch_sweep_tb(c->cfg, c->args(parity), c->work));
    else HIPCHK(launch_sweep(c->cfg, c->args(parity), c->work));
    if (c->timing) HIPCHK(hipEventRecord(c->ev_pool[c->ev_used++], c->work));
    return GLBM_OK;
}

int upload_state(glbm_ctx c)
{
    HIPCHK(hipMemcpyAsync(c->inst_d, c->inst_h.data(), c->inst_h.size() * sizeof(InstDev), hipMemcpyHostToDevice,
                          c->work));
    HIPCHK(hipMemcpyAsync(c->active_d, c->active_h.data(), c->active_h.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, c->work));
    HIPCHK(hipMemcpyAsync(c->dsteps_d, c->dsteps_h.data(), c->dsteps_h.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, c->work));
    // the host vectors may change before the copies run
    HIPCHK(hipStreamSynchronize(c->work));
    return GLBM_OK;
}

// Observe the current state of every instance (snapshot u) without a residual.
int take_snapshot(glbm_ctx c)
{
    HIPCHK(launch_observe(c->cfg, c->args(c->gstep), 1 | 4, c->work));
    for (int i = 0; i < c->n_inst; ++i) c->snap_step[i] = c->steps[i];
    c->snap_valid = true;
    return GLBM_OK;
}

int capture_chunk(glbm_ctx c, double tol)
{
    free_graph(c);
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->work, hipStreamCaptureModeRelaxed));
    hipError_t err = hipSuccess;
    // chunks start at an even global step (n_c is even)
    const int two = c->tb_on() ? c->n_c / 4 * 2 : 0;
    for (int j = 0; j < two && err == hipSuccess; ++j) err = launch_sweep_tb(c->cfg, c->args(j), c->work);
    for (int k = 2 * two; k < c->n_c && err == hipSuccess; ++k) err = launch_sweep(c->cfg, c->args(k), c->work);
    if (err == hipSuccess) err = launch_observe(c->cfg, c->args(0), 3, c->work);
    if (err == hipSuccess) err = launch_finalize(c->args(0), c->n_inst, tol, 1, 1, c->work);
    hipError_t e2 = hipStreamEndCapture(c->work, &g);
    if (err != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(GLBM_EDEVICE, "graph capture: %s", hipGetErrorString(err));
    }
    HIPCHK(e2);
    err = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (err != hipSuccess) {
        c->graph = nullptr;
        return fail(GLBM_EDEVICE, "graph instantiate: %s", hipGetErrorString(err));
    }
    c->graph_tol = tol;
    c->graph_valid = true;
    return GLBM_OK;
}

int check_tables(glbm_ctx c)
{
    for (int i = 0; i < c->n_inst; ++i)
        if (!c->has_table[i]) return fail(GLBM_ESTATE, "instance %d: glbm_set_local_perm not called", i);
    return GLBM_OK;
}

void set_parities(glbm_ctx c)
{
    for (int i = 0; i < c->n_inst; ++i) c->inst_h[i].par = (int32_t)((c->steps[i] - c->gstep) & 1);
}

// Copy one instance's class table (kClasses x kTabW doubles) to the device in the compute type.
int upload_table(glbm_ctx c, int inst, const std::vector<double>& row)
{
    char* dst = static_cast<char*>(c->tab_d) + (size_t)inst * kClasses * kTabW * c->tsz;
    if (c->tsz == 8) {
        HIPCHK(hipMemcpyAsync(dst, row.data(), row.size() * 8, hipMemcpyHostToDevice, c->work));
    } else {
        std::vector<float> rf(row.begin(), row.end());
        HIPCHK(hipMemcpyAsync(dst, rf.data(), rf.size() * 4, hipMemcpyHostToDevice, c->work));
    }
    HIPCHK(hipStreamSynchronize(c->work));
    return GLBM_OK;
}

int read_results(glbm_ctx c)
{
    HIPCHK(hipMemcpyAsync(c->res_p, c->res_d, (size_t)c->n_inst * kResW * sizeof(double), hipMemcpyDeviceToHost,
                          c->work));
    HIPCHK(hipMemcpyAsync(c->active_p, c->active_d, (size_t)c->n_inst * sizeof(int32_t), hipMemcpyDeviceToHost,
                          c->work));
    HIPCHK(hipStreamSynchronize(c->work));
    return GLBM_OK;
}

}  // namespace

extern "C" {

const char* glbm_last_error(void) { return g_err.c_str(); }

size_t glbm_required_bytes(int32_t n_inst, const glbm_instance_desc* desc)
{
    if (validate(n_inst, desc) != GLBM_OK) return 0;
    Layout L = layout_of(n_inst, desc);
    const size_t one = (size_t)round_up(L.elems * (int64_t)store_bytes(desc[0].store), 256);
    return 2 * one;
}

int glbm_init_geometry(glbm_ctx* out, int32_t n_inst, const glbm_instance_desc* desc, const uint8_t* const* cls_host,
                       void* pop_dev, size_t pop_bytes, void* hip_stream)
{
    g_err.clear();
    if (!out) return fail(GLBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(n_inst, desc);
    if (rc) return rc;
    if (!cls_host) return fail(GLBM_EINVAL, "cls_host is NULL");
    for (int i = 0; i < n_inst; ++i)
        if (!cls_host[i]) return fail(GLBM_EINVAL, "cls_host[%d] is NULL", i);
    const size_t need = glbm_required_bytes(n_inst, desc);
    if (pop_dev && pop_bytes < need)
        return fail(GLBM_ENOMEM, "population buffer too small: %zu < %zu bytes", pop_bytes, need);
    if (pop_dev && reinterpret_cast<uintptr_t>(pop_dev) % 256)
        return fail(GLBM_EINVAL, "population buffer must be 256-byte aligned");

    glbm_ctx c = new (std::nothrow) glbm_ctx_s();
    if (!c) return fail(GLBM_ENOMEM, "host allocation failed");
    c->n_inst = n_inst;
    c->desc.assign(desc, desc + n_inst);
    c->cfg.q = desc[0].lattice;
    c->cfg.store = desc[0].store;
    c->cfg.forch = false;
    c->n_c = desc[0].check_every;
    c->esz = store_bytes(desc[0].store);
    c->tsz = compute_bytes(desc[0].store);
    c->user = static_cast<hipStream_t>(hip_stream);

    auto bail = [&](int code) {
        glbm_destroy(c);
        return code;
    };
#define TRY(expr)                        \
    do {                                 \
        int r_ = (expr);                 \
        if (r_) return bail(r_);         \
    } while (0)
#define TRYHIP(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return bail(fail(e_ == hipErrorOutOfMemory ? GLBM_ENOMEM : GLBM_EDEVICE, \
                                               "%s failed: %s", #expr, hipGetErrorString(e_)));    \
    } while (0)

    TRYHIP(hipGetDevice(&c->device));
    TRY(fetch_scratch(c->device));
    TRYHIP(hipStreamCreateWithFlags(&c->work, hipStreamDefault));
    TRYHIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    TRYHIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));

    Layout L = layout_of(n_inst, desc);
    int64_t cls_total = 0, snap_total = 0;
    bool any_wall_node = false, any_wall_face = false;
    c->cls_h.resize(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const glbm_instance_desc& d = desc[i];
        const int64_t n = (int64_t)d.nx * d.ny * d.nz;
        InstDev I{};
        I.pop_off = L.off[i];
        I.cls_off = cls_total;
        I.snap_off = snap_total;
        I.stride = (int32_t)L.stride[i];
        I.nx = d.nx;
        I.ny = d.ny;
        I.nz = d.nz;
        I.walls = d.wall_faces;
        I.par = 0;
        for (int a = 0; a < 3; ++a) I.g[a] = d.g[a];
        I.omega = 1.0 / d.tau;
        I.cforce = 1.0 - 0.5 / d.tau;
        I.nu = (d.tau - 0.5) / 3.0;
        for (int a = 0; a < 3; ++a) I.gf[a] = (float)I.g[a];
        I.omegaf = (float)I.omega;
        I.cforcef = (float)I.cforce;
        const bool half = d.store == GLBM_STORE_F16DEV || d.store == GLBM_STORE_F16LOC;
        const int s = half ? (d.dev_scale_log2 == GLBM_SCALE_AUTO ? auto_scale(d) : d.dev_scale_log2) : 0;
        I.scale = std::ldexp(1.0f, s);
        I.inv_scale = std::ldexp(1.0f, -s);
        I.paxis = d.pressure_axis ? d.pressure_axis - 1 : 0;
        I.drin = d.pressure_axis ? d.rho_in - 1.0 : 0.0;
        I.drout = d.pressure_axis ? d.rho_out - 1.0 : 0.0;
        I.p0 = 1.0;   // pressure map: set by glbm_set_pressure_perm (unused by a constant K)
        I.p1 = 0.0;
        I.drinf = (float)I.drin;
        I.droutf = (float)I.drout;
        I.p0f = (float)I.p0;
        I.p1f = (float)I.p1;
        I.nuf = (float)I.nu;
        c->inst_h.push_back(I);
        c->cls_h[i].assign(cls_host[i], cls_host[i] + n);
        int64_t nf = 0;
        for (int64_t k = 0; k < n; ++k) {
            if (cls_host[i][k] == kWallClass) any_wall_node = true;
            else ++nf;
        }
        if (nf == 0) return bail(fail(GLBM_EINVAL, "instance %d has no fluid node", i));
        c->n_fluid.push_back(nf);
        if (d.wall_faces) any_wall_face = true;
        cls_total += round_up(n, 256);
        snap_total += round_up(3 * n, 64);
    }
    c->cfg.bc = desc[0].pressure_axis ? (any_wall_node ? 4 : 3) : (any_wall_node ? 2 : (any_wall_face ? 1 : 0));
    c->staged_ok = c->cfg.q == GLBM_D2Q9 && c->cfg.bc == 0 &&
                   (c->cfg.store == GLBM_STORE_F16DEV || c->cfg.store == GLBM_STORE_F16LOC);
    for (int i = 0; i < n_inst; ++i)
        if (desc[i].nx % 8) c->staged_ok = false;
    c->paired_ok = c->cfg.q == GLBM_D2Q9 && c->cfg.bc == 0 &&
                   (c->cfg.store == GLBM_STORE_F16DEV || c->cfg.store == GLBM_STORE_F16LOC);
    for (int i = 0; i < n_inst; ++i)
        if (desc[i].nx % 2) c->paired_ok = false;
    c->steps.assign(n_inst, 0);
    c->snap_step.assign(n_inst, 0);
    c->active_h.assign(n_inst, 1);
    c->dsteps_h.assign(n_inst, c->n_c);
    c->has_table.assign(n_inst, 0);
    c->eps_h.assign(n_inst, std::vector<double>(kClasses, 1.0));
    c->k_h.assign(n_inst, std::vector<double>(kClasses, INFINITY));
    c->snap_elems = snap_total;

    // population buffers
    const size_t half = need / 2;
    if (pop_dev) {
        c->pop_base = pop_dev;
        c->own_pop = false;
    } else {
        TRYHIP(hipMalloc(&c->pop_base, need));
        c->own_pop = true;
    }
    c->pop_bytes = need;
    c->buf[0] = c->pop_base;
    c->buf[1] = static_cast<char*>(c->pop_base) + half;

    TRYHIP(hipMalloc(&c->cls_d, (size_t)cls_total));
    TRYHIP(hipMalloc(&c->inst_d, n_inst * sizeof(InstDev)));
    TRYHIP(hipMalloc(&c->tab_d, (size_t)n_inst * kClasses * kTabW * c->tsz));
    TRYHIP(hipMalloc(&c->snap_d, (size_t)snap_total * c->tsz));
    TRYHIP(hipMalloc(&c->res_d, (size_t)n_inst * kResW * sizeof(double)));
    TRYHIP(hipMalloc(&c->flux_d, (size_t)n_inst * kResW * sizeof(double)));
    TRYHIP(hipMalloc(&c->active_d, n_inst * sizeof(int32_t)));
    TRYHIP(hipMalloc(&c->dsteps_d, n_inst * sizeof(int32_t)));
    TRYHIP(hipHostMalloc(reinterpret_cast<void**>(&c->res_p), (size_t)n_inst * kResW * sizeof(double),
                         hipHostMallocDefault));
    TRYHIP(hipHostMalloc(reinterpret_cast<void**>(&c->active_p), n_inst * sizeof(int32_t), hipHostMallocDefault));

    TRY(enter(c));
    for (int i = 0; i < n_inst; ++i)
        TRYHIP(hipMemcpyAsync(c->cls_d + c->inst_h[i].cls_off, c->cls_h[i].data(), c->cls_h[i].size(),
                              hipMemcpyHostToDevice, c->work));
    // rest state: all deviations zero (f_i = w_i, rho = 1, u = 0)
    TRYHIP(launch_zero(c->pop_base, need, c->work));
    TRYHIP(launch_zero(c->snap_d, (size_t)snap_total * c->tsz, c->work));
    TRYHIP(launch_zero(c->res_d, (size_t)n_inst * kResW * sizeof(double), c->work));
    TRYHIP(launch_zero(c->tab_d, (size_t)n_inst * kClasses * kTabW * c->tsz, c->work));
    for (int i = 0; i < n_inst; ++i) c->res_p[i * kResW + P_R] = INFINITY;
    default_tile(c);
    TRY(build_tiles(c));
    TRY(upload_state(c));
    TRY(leave(c));
    *out = c;
    return GLBM_OK;
#undef TRY
#undef TRYHIP
}

int glbm_set_local_perm(glbm_ctx c, int32_t inst, int32_t n_classes, const double* eps, const double* k_lattice,
                        const double* f_eps)
{
    g_err.clear();
    if (!c) return fail(GLBM_EINVAL, "null context");
    if (inst < -1 || inst >= c->n_inst) return fail(GLBM_EINVAL, "instance %d out of range", inst);
    if (n_classes < 1 || n_classes > 255) return fail(GLBM_EINVAL, "n_classes must be in [1, 255]");
    if (!eps || !k_lattice) return fail(GLBM_EINVAL, "eps and k_lattice are required");
    for (int k = 0; k < n_classes; ++k) {
        if (!(eps[k] > 0.0 && eps[k] <= 1.0)) return fail(GLBM_EINVAL, "class %d: eps %g outside (0, 1]", k, eps[k]);
        if (!(k_lattice[k] > 0.0)) return fail(GLBM_EINVAL, "class %d: K %g must be > 0", k, k_lattice[k]);
        if (f_eps && !(f_eps[k] >= 0.0 && std::isfinite(f_eps[k])))
            return fail(GLBM_EINVAL, "class %d: F_eps %g must be finite and >= 0", k, f_eps[k]);
    }
    const int i0 = inst < 0 ? 0 : inst, i1 = inst < 0 ? c->n_inst : inst + 1;
    for (int i = i0; i < i1; ++i)
        for (uint8_t v : c->cls_h[i])
            if (v != kWallClass && v >= n_classes)
                return fail(GLBM_EINVAL, "instance %d: class %d of the map has no table entry", i, (int)v);
    bool forch = false;
    for (int k = 0; k < n_classes && f_eps; ++k)
        if (f_eps[k] > 0.0 && std::isfinite(k_lattice[k])) forch = true;
    if (forch && c->cfg.bc >= 3) return fail(GLBM_EINVAL, "F_eps > 0 is not supported with pressure faces");

    int rc = enter(c);
    if (rc) return rc;
    Joined joined(c);
    std::vector<double> row((size_t)kClasses * kTabW, 0.0);
    for (int i = i0; i < i1; ++i) {
        const double nu = c->inst_h[i].nu;
        std::fill(row.begin(), row.end(), 0.0);
        for (int k = 0; k < kClasses; ++k) {
            const bool have = k < n_classes;
            const double e = have ? eps[k] : 1.0;
            const double kinv = (have && std::isfinite(k_lattice[k])) ? 1.0 / k_lattice[k] : 0.0;
            const double fe = (have && f_eps) ? f_eps[k] : 0.0;
            const double c0 = 0.5 * (1.0 + e * 0.5 * nu * kinv);   // Eq. (36)
            const double c1 = e * 0.5 * fe * std::sqrt(kinv);      // Eq. (37)
            double* r = &row[(size_t)k * kTabW];
            r[TAB_EPS] = e;
            r[TAB_INV_EPS] = 1.0 / e;
            if (c->cfg.bc >= 3) {
                // pressure-driven format with a pressure-independent K: K(P) = A
                const bool open = kinv == 0.0;
                r[TAB_PA] = open ? 1.0 : k_lattice[k];
                r[TAB_PB] = r[TAB_PC] = r[TAB_PBL] = 0.0;
                r[TAB_POPEN] = open ? 0.0 : 1.0;
                continue;
            }
            r[TAB_INV_2C0] = 1.0 / (2.0 * c0);
            r[TAB_DRAG] = e * nu * kinv;
            r[TAB_C0] = c0;
            r[TAB_C1] = c1;
            r[TAB_FORCH] = e * fe * std::sqrt(kinv);
        }
        int rc2 = upload_table(c, i, row);
        if (rc2) return rc2;
        c->has_table[i] = 1;
        for (int k = 0; k < n_classes; ++k) {
            c->eps_h[i][k] = eps[k];
            c->k_h[i][k] = k_lattice[k];
        }
    }
    if (forch && !c->cfg.forch) {
        c->cfg.forch = true;
        free_graph(c);
    }
    c->snap_valid = false;
    free_graph(c);
    return joined.done();
}

int glbm_set_pressure_perm(glbm_ctx c, int32_t inst, int32_t n_classes, const double* eps, const double* k_const,
                           const double* k_kn, const double* k_surf, const double* lb, double p_in, double p_out)
{
    g_err.clear();
    if (!c) return fail(GLBM_EINVAL, "null context");
    if (c->cfg.bc < 3) return fail(GLBM_EINVAL, "the instances of this context have no pressure faces");
    if (inst < -1 || inst >= c->n_inst) return fail(GLBM_EINVAL, "instance %d out of range", inst);
    if (n_classes < 1 || n_classes > 255) return fail(GLBM_EINVAL, "n_classes must be in [1, 255]");
    if (!eps || !k_const || !k_kn || !k_surf || !lb) return fail(GLBM_EINVAL, "every coefficient array is required");
    if (!(p_in > 0.0) || !(p_out > 0.0) || !std::isfinite(p_in) || !std::isfinite(p_out))
        return fail(GLBM_EINVAL, "p_in and p_out must be finite and > 0");
    const double plo = std::min(p_in, p_out), phi = std::max(p_in, p_out);
    for (int k = 0; k < n_classes; ++k) {
        if (!(eps[k] > 0.0 && eps[k] <= 1.0)) return fail(GLBM_EINVAL, "class %d: eps %g outside (0, 1]", k, eps[k]);
        if (!(k_const[k] > 0.0)) return fail(GLBM_EINVAL, "class %d: k_const %g must be > 0", k, k_const[k]);
        if (std::isinf(k_const[k])) continue;
        if (!(k_kn[k] >= 0.0) || !(k_surf[k] >= 0.0) || !(lb[k] >= 0.0) || !std::isfinite(k_kn[k]) ||
            !std::isfinite(k_surf[k]) || !std::isfinite(lb[k]))
            return fail(GLBM_EINVAL, "class %d: k_knudsen, k_surface and langmuir_b must be finite and >= 0", k);
        for (double P : {plo, phi}) {
            const double K = k_const[k] + (k_kn[k] + k_surf[k] / (1.0 + lb[k] * P)) / P;
            if (!(K > 0.0) || !std::isfinite(K)) return fail(GLBM_EINVAL, "class %d: K(%g) = %g", k, P, K);
        }
    }
    const int i0 = inst < 0 ? 0 : inst, i1 = inst < 0 ? c->n_inst : inst + 1;
    for (int i = i0; i < i1; ++i)
        for (uint8_t v : c->cls_h[i])
            if (v != kWallClass && v >= n_classes)
                return fail(GLBM_EINVAL, "instance %d: class %d of the map has no table entry", i, (int)v);
    int rc = enter(c);
    if (rc) return rc;
    Joined joined(c);
    std::vector<double> row((size_t)kClasses * kTabW, 0.0);
    for (int i = i0; i < i1; ++i) {
        std::fill(row.begin(), row.end(), 0.0);
        for (int k = 0; k < kClasses; ++k) {
            const bool have = k < n_classes;
            const bool open = !have || std::isinf(k_const[k]);
            double* r = &row[(size_t)k * kTabW];
            r[TAB_EPS] = have ? eps[k] : 1.0;
            r[TAB_INV_EPS] = 1.0 / r[TAB_EPS];
            r[TAB_PA] = open ? 1.0 : k_const[k];
            r[TAB_PB] = open ? 0.0 : k_kn[k];
            r[TAB_PC] = open ? 0.0 : k_surf[k];
            r[TAB_PBL] = open ? 0.0 : lb[k];
            r[TAB_POPEN] = open ? 0.0 : 1.0;
        }
        rc = upload_table(c, i, row);
        if (rc) return rc;
        InstDev& I = c->inst_h[i];
        const glbm_instance_desc& d = c->desc[i];
        // P = p_out + (rho - rho_out) (p_in - p_out) / (rho_in - rho_out) = p0 + (rho - 1) p1
        I.p1 = (p_in - p_out) / (d.rho_in - d.rho_out);
        I.p0 = p_out - (d.rho_out - 1.0) * I.p1;
        I.p0f = (float)I.p0;
        I.p1f = (float)I.p1;
        c->has_table[i] = 1;
        for (int k = 0; k < n_classes; ++k) {
            c->eps_h[i][k] = eps[k];
            c->k_h[i][k] = k_const[k];
        }
    }
    rc = upload_state(c);
    if (rc) return rc;
    c->snap_valid = false;
    free_graph(c);
    return joined.done();
}

int glbm_step_n(glbm_ctx c, int64_t n, double tol)
{
    g_err.clear();
    if (!c) return fail(GLBM_EINVAL, "null context");
    if (n < 0) return fail(GLBM_EINVAL, "n must be >= 0");
    int rc = check_tables(c);
    if (rc) return rc;
    rc = enter(c);
    if (rc) return rc;
    Joined joined(c);

    // (re)activate: everything when tol <= 0, else every instance not already below tol
    for (int i = 0; i < c->n_inst; ++i) {
        const double r = c->res_p[i * kResW + P_R];
        c->active_h[i] = (tol > 0.0 && c->snap_valid && r <= tol && c->snap_step[i] == c->steps[i]) ? 0 : 1;
    }
    set_parities(c);
    rc = upload_state(c);
    if (rc) return rc;
    if (!c->snap_valid) {
        rc = take_snapshot(c);
        if (rc) return rc;
    }
    bool nonfinite = false;
    int unstable = -1;  // first instance whose check saw |u| > kUMax
    int64_t left = n;
    auto any_active = [&]() {
        for (int i = 0; i < c->n_inst; ++i)
            if (c->active_h[i]) return true;
        return false;
    };
    while (left > 0 && any_active()) {
        const int64_t phase = c->gstep % c->n_c;
        const int64_t len = std::min<int64_t>(c->n_c - phase, left);
        const bool check = phase + len == c->n_c;
        if (check) {
            // steps since each active instance's snapshot, after this chunk
            bool changed = false;
            for (int i = 0; i < c->n_inst; ++i) {
                if (!c->active_h[i]) continue;
                const int32_t ds = (int32_t)(c->steps[i] + len - c->snap_step[i]);
                if (ds != c->dsteps_h[i]) changed = true;
                c->dsteps_h[i] = ds;
            }
            if (changed) {
                rc = upload_state(c);
                if (rc) return rc;
            }
        }
        if (check && len == c->n_c && c->use_graph && !c->timing && (c->gstep & 1) == 0) {
            if (!c->graph_valid || c->graph_tol != tol) {
                rc = capture_chunk(c, tol);
                if (rc) return rc;
            }
            HIPCHK(hipGraphLaunch(c->graph, c->work));
        } else {
            int64_t k = 0;
            if (c->tb_on() && (c->gstep & 1) == 0) {
                const int64_t two = len / 4 * 2;
                for (int64_t j = 0; j < two; ++j) {
                    rc = sweep_once(c, (int)((c->gstep + j) & 1), true);
                    if (rc) return rc;
                }
                k = 2 * two;
            }
            for (; k < len; ++k) {
                rc = sweep_once(c, (int)((c->gstep + k) & 1));
                if (rc) return rc;
            }
            if (check) {
                HIPCHK(launch_observe(c->cfg, c->args(c->gstep + len), 3, c->work));
                HIPCHK(launch_finalize(c->args(c->gstep + len), c->n_inst, tol, 1, 1, c->work));
            }
        }
        c->gstep += len;
        left -= len;
        for (int i = 0; i < c->n_inst; ++i)
            if (c->active_h[i]) c->steps[i] += len;
        if (check) {
            rc = read_results(c);
            if (rc) return rc;
            for (int i = 0; i < c->n_inst; ++i) {
                if (!c->active_h[i]) continue;
                c->snap_step[i] = c->steps[i];
                if (!std::isfinite(c->res_p[i * kResW + P_R]) && c->res_p[i * kResW + P_BAD] > 0) nonfinite = true;
                if (c->res_p[i * kResW + P_FAST] > 0 && unstable < 0) unstable = i;
                c->active_h[i] = c->active_p[i];
            }
            if (nonfinite || unstable >= 0) break;
        }
    }
    if (c->timing) {
        rc = resolve_timing(c);
        if (rc) return rc;
    }
    // host view of the active flags may differ from the device after the loop; keep them equal
    set_parities(c);
    rc = upload_state(c);
    if (rc) return rc;
    rc = joined.done();
    if (rc) return rc;
    if (nonfinite) return fail(GLBM_ENONFINITE, "non-finite populations detected");
    if (unstable >= 0)
        return fail(GLBM_EUNSTABLE, "instance %d: %.0f nodes with |u| > %g at step %lld (outside the low-Mach range)",
                    unstable, c->res_p[unstable * kResW + P_FAST], kUMax, (long long)c->steps[unstable]);
    if (tol > 0.0 && any_active()) return fail(GLBM_ENOTCONVERGED, "step budget reached before r <= %g", tol);
    return GLBM_OK;
}

int glbm_residual(glbm_ctx c, double* r, int64_t* steps)
{
    g_err.clear();
    if (!c) return fail(GLBM_EINVAL, "null context");
    HIPCHK(hipStreamSynchronize(c->work));
    for (int i = 0; i < c->n_inst; ++i) {
        if (r) r[i] = c->res_p[i * kResW + P_R];
        if (steps) steps[i] = c->steps[i];
    }
    return GLBM_OK;
}

int glbm_permeability(glbm_ctx c, double* k)
{
    g_err.clear();
    if (!c) return fail(GLBM_EINVAL, "null context");
    if (!k) return fail(GLBM_EINVAL, "k is NULL");
    int rc = check_tables(c);
    if (rc) return rc;
    rc = enter(c);
    if (rc) return rc;
    Joined joined(c);
    Args a = c->args(c->gstep);
    a.res = c->flux_d;
    HIPCHK(launch_observe(c->cfg, a, 4, c->work));
    HIPCHK(launch_finalize(a, c->n_inst, 0.0, 0, 0, c->work));
    std::vector<double> h((size_t)c->n_inst * kResW);
    HIPCHK(hipMemcpyAsync(h.data(), c->flux_d, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->work));
    HIPCHK(hipStreamSynchronize(c->work));
    for (int i = 0; i < c->n_inst; ++i) {
        const double nu = c->inst_h[i].nu;
        const glbm_instance_desc& D = c->desc[i];
        for (int d = 0; d < 3; ++d) {
            const double g = c->inst_h[i].g[d];
            const double mean = h[i * kResW + P_UX + d] / (double)c->n_fluid[i];
            k[3 * i + d] = g != 0.0 ? nu * mean / g : NAN;
            if (D.pressure_axis == d + 1) {
                // Darcy's law with the lattice pressure c_s^2 rho across the n - 1 node spacings between the faces
                const int32_t na = d == 0 ? D.nx : (d == 1 ? D.ny : D.nz);
                k[3 * i + d] = nu * mean * (double)(na - 1) / ((D.rho_in - D.rho_out) / 3.0);
            }
        }
    }
    return joined.done();
}

static int set_fields_impl(glbm_ctx c, int32_t inst, const void* rho_d, const void* u_d, int is_double)
{
    HIPCHK(launch_set_fields(c->cfg, c->args(c->gstep), inst, c->inst_h[inst].ntiles, rho_d, u_d, is_double,
                             c->work));
    c->snap_valid = false;
    for (int i = 0; i < c->n_inst; ++i) c->res_p[i * kResW + P_R] = INFINITY;
    HIPCHK(hipMemcpyAsync(c->res_d, c->res_p, (size_t)c->n_inst * kResW * sizeof(double), hipMemcpyHostToDevice,
                          c->work));
    HIPCHK(hipStreamSynchronize(c->work));
    return GLBM_OK;
}

int glbm_set_fields(glbm_ctx c, int32_t inst, const double* rho, const double* u)
{
    g_err.clear();
    if (!c) return fail(GLBM_EINVAL, "null context");
    if (inst < 0 || inst >= c->n_inst) return fail(GLBM_EINVAL, "instance %d out of range", inst);
    if (!rho || !u) return fail(GLBM_EINVAL, "rho and u are required");
    int rc = check_tables(c);
    if (rc) return rc;
    rc = enter(c);
    if (rc) return rc;
    Joined joined(c);
    const InstDev& I = c->inst_h[inst];
    const size_t n = (size_t)I.nx * I.ny * I.nz;
    double* d = nullptr;
    HIPCHK(hipMalloc(&d, 4 * n * sizeof(double)));
    hipError_t e = hipMemcpyAsync(d, rho, n * sizeof(double), hipMemcpyHostToDevice, c->work);
    if (e == hipSuccess) e = hipMemcpyAsync(d + n, u, 3 * n * sizeof(double), hipMemcpyHostToDevice, c->work);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail(GLBM_EDEVICE, "upload: %s", hipGetErrorString(e));
    }
    rc = set_fields_impl(c, inst, d, d + n, 1);
    hipError_t es = hipStreamSynchronize(c->work);
    (void)hipFree(d);
    if (rc) return rc;
    HIPCHK(es);
    return joined.done();
}

int glbm_set_fields_device(glbm_ctx c, int32_t inst, const float* drho_dev, const float* u_dev)
{
    g_err.clear();
    if (!c) return fail(GLBM_EINVAL, "null context");
    if (inst < 0 || inst >= c->n_inst) return fail(GLBM_EINVAL, "instance %d out of range", inst);
    if (!drho_dev || !u_dev) return fail(GLBM_EINVAL, "drho and u are required");
    int rc = check_tables(c);
    if (rc) return rc;
    rc = enter(c);
    if (rc) return rc;
    Joined joined(c);
    rc = set_fields_impl(c, inst, drho_dev, u_dev, 0);
    if (rc) return rc;
    return joined.done();
}

static int get_impl(glbm_ctx c, int32_t inst, double* rho, double* u, double* pops)
{
    if (!c) return fail(GLBM_EINVAL, "null context");
    if (inst < 0 || inst >= c->n_inst) return fail(GLBM_EINVAL, "instance %d out of range", inst);
    int rc = check_tables(c);
    if (rc) return rc;
    rc = enter(c);
    if (rc) return rc;
    Joined joined(c);
    const InstDev& I = c->inst_h[inst];
    const size_t n = (size_t)I.nx * I.ny * I.nz;
    const size_t q = (size_t)c->cfg.q;
    double* d = nullptr;
    HIPCHK(hipMalloc(&d, (4 + q) * n * sizeof(double)));
    hipError_t e = launch_get_fields(c->cfg, c->args(c->gstep), inst, I.ntiles, d, d + n, pops ? d + 4 * n : nullptr,
                                     c->work);
    if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, d, n * sizeof(double), hipMemcpyDeviceToHost, c->work);
    if (e == hipSuccess && u) e = hipMemcpyAsync(u, d + n, 3 * n * sizeof(double), hipMemcpyDeviceToHost, c->work);
    if (e == hipSuccess && pops)
        e = hipMemcpyAsync(pops, d + 4 * n, q * n * sizeof(double), hipMemcpyDeviceToHost, c->work);
    hipError_t es = hipStreamSynchronize(c->work);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(GLBM_EDEVICE, "get fields: %s", hipGetErrorString(e));
    HIPCHK(es);
    return joined.done();
}

int glbm_get_fields(glbm_ctx c, int32_t inst, double* rho, double* u)
{
    g_err.clear();
    return get_impl(c, inst, rho, u, nullptr);
}

int glbm_get_populations(glbm_ctx c, int32_t inst, double* f_host)
{
    g_err.clear();
    if (!f_host) return fail(GLBM_EINVAL, "f_host is NULL");
    return get_impl(c, inst, nullptr, nullptr, f_host);
}

// checkpoint layout: header | populations (both buffers) | snapshots | results | counters
struct CkptHeader {
    uint64_t magic, pop_bytes, snap_bytes, n_inst;
    int64_t gstep;
    int32_t snap_valid, pad;
};
static const uint64_t kMagic = 0x474c424d434b5031ULL;

size_t glbm_state_bytes(glbm_ctx c)
{
    if (!c) return 0;
    return sizeof(CkptHeader) + c->pop_bytes + (size_t)c->snap_elems * c->tsz +
           (size_t)c->n_inst * (kResW * sizeof(double) + 2 * sizeof(int64_t));
}

int glbm_save_state(glbm_ctx c, void* host, size_t bytes)
{
    g_err.clear();
    if (!c || !host) return fail(GLBM_EINVAL, "null argument");
    if (bytes < glbm_state_bytes(c)) return fail(GLBM_ENOMEM, "buffer too small");
    int rc = enter(c);
    if (rc) return rc;
    Joined joined(c);
    char* p = static_cast<char*>(host);
    CkptHeader h{kMagic, c->pop_bytes, (uint64_t)c->snap_elems * c->tsz, (uint64_t)c->n_inst, c->gstep,
                 c->snap_valid ? 1 : 0, 0};
    memcpy(p, &h, sizeof h);
    p += sizeof h;
    HIPCHK(hipMemcpyAsync(p, c->pop_base, c->pop_bytes, hipMemcpyDeviceToHost, c->work));
    p += c->pop_bytes;
    HIPCHK(hipMemcpyAsync(p, c->snap_d, h.snap_bytes, hipMemcpyDeviceToHost, c->work));
    p += h.snap_bytes;
    HIPCHK(hipStreamSynchronize(c->work));
    memcpy(p, c->res_p, (size_t)c->n_inst * kResW * sizeof(double));
    p += (size_t)c->n_inst * kResW * sizeof(double);
    memcpy(p, c->steps.data(), c->n_inst * sizeof(int64_t));
    p += c->n_inst * sizeof(int64_t);
    memcpy(p, c->snap_step.data(), c->n_inst * sizeof(int64_t));
    return joined.done();
}

int glbm_load_state(glbm_ctx c, const void* host, size_t bytes)
{
    g_err.clear();
    if (!c || !host) return fail(GLBM_EINVAL, "null argument");
    if (bytes < glbm_state_bytes(c)) return fail(GLBM_EINVAL, "checkpoint too small");
    const char* p = static_cast<const char*>(host);
    CkptHeader h;
    memcpy(&h, p, sizeof h);
    if (h.magic != kMagic || h.pop_bytes != c->pop_bytes || h.n_inst != (uint64_t)c->n_inst ||
        h.snap_bytes != (uint64_t)c->snap_elems * c->tsz)
        return fail(GLBM_EINVAL, "checkpoint does not match this context");
    int rc = enter(c);
    if (rc) return rc;
    Joined joined(c);
    p += sizeof h;
    HIPCHK(hipMemcpyAsync(c->pop_base, p, c->pop_bytes, hipMemcpyHostToDevice, c->work));
    p += c->pop_bytes;
    HIPCHK(hipMemcpyAsync(c->snap_d, p, h.snap_bytes, hipMemcpyHostToDevice, c->work));
    p += h.snap_bytes;
    HIPCHK(hipStreamSynchronize(c->work));
    memcpy(c->res_p, p, (size_t)c->n_inst * kResW * sizeof(double));
    p += (size_t)c->n_inst * kResW * sizeof(double);
    memcpy(c->steps.data(), p, c->n_inst * sizeof(int64_t));
    p += c->n_inst * sizeof(int64_t);
    memcpy(c->snap_step.data(), p, c->n_inst * sizeof(int64_t));
    c->gstep = h.gstep;
    c->snap_valid = h.snap_valid != 0;
    HIPCHK(hipMemcpyAsync(c->res_d, c->res_p, (size_t)c->n_inst * kResW * sizeof(double), hipMemcpyHostToDevice,
                          c->work));
    set_parities(c);
    rc = upload_state(c);
    if (rc) return rc;
    free_graph(c);
    return joined.done();
}

int glbm_set_option(glbm_ctx c, int32_t option, int64_t value)
{
    g_err.clear();
    if (!c) return fail(GLBM_EINVAL, "null context");
    switch (option) {
    case GLBM_OPT_GRAPH:
        c->use_graph = value != 0;
        return GLBM_OK;
    case GLBM_OPT_TIMING: {
        int rc = resolve_timing(c);
        if (rc) return rc;
        c->timing = value != 0;
        c->time_ms = 0.0;
        c->launches = 0;
        return GLBM_OK;
    }
    case GLBM_OPT_TILE_ROWS:
    case GLBM_OPT_TILE_WIDTH: {
        int twl = c->tw_log2, th = c->th;
        if (option == GLBM_OPT_TILE_ROWS) {
            th = (int)value;
        } else {
            int l = 6;
            while (l <= 10 && (1 << l) != value) ++l;
            if (l > 10) return fail(GLBM_EINVAL, "tile width must be a power of two in [64, 1024]");
            twl = l;
            if (((1 << twl) * th) % kBlock) th = kBlock >> twl;
        }
        if (!tile_ok(twl, th))
            return fail(GLBM_EINVAL, "tile %d x %d must hold a multiple of %d nodes (height 1..256)", 1 << twl, th,
                        kBlock);
        if (twl == c->tw_log2 && th == c->th) return GLBM_OK;
        HIPCHK(hipStreamSynchronize(c->work));
        c->tw_log2 = twl;
        c->th = th;
        return build_tiles(c);
    }
    case GLBM_OPT_CACHE:
        if (value < 0 || value > 127) return fail(GLBM_EINVAL, "memory policy must be in [0, 127]");
        c->cache = (int)value;
        free_graph(c);
        return GLBM_OK;
    default:
        return fail(GLBM_EINVAL, "unknown option %d", option);
    }
}

int glbm_sweep_time(glbm_ctx c, double* ms_total, int64_t* launches)
{
    g_err.clear();
    if (!c) return fail(GLBM_EINVAL, "null context");
    int rc = resolve_timing(c);
    if (rc) return rc;
    if (ms_total) *ms_total = c->time_ms;
    if (launches) *launches = c->launches;
    return GLBM_OK;
}

int glbm_sweeps_per_launch(glbm_ctx c, int32_t* sweeps)
{
    g_err.clear();
    if (!c || !sweeps) return fail(GLBM_EINVAL, "null context or output");
    *sweeps = c->tb_on() ? 2 : 1;
    return GLBM_OK;
}

int glbm_autotune(glbm_ctx c, int32_t steps, int32_t* chosen)
{
    g_err.clear();
    if (!c) return fail(GLBM_EINVAL, "null context");
    if (steps < 2 || (steps & 1)) return fail(GLBM_EINVAL, "steps must be even and >= 2");
    int rc = check_tables(c);
    if (rc) return rc;
    const bool old_timing = c->timing;
    int max_nx = 1;
    for (auto& I : c->inst_h) max_nx = std::max(max_nx, I.nx);
    double best = 1e300;
    int best_twl = c->tw_log2, best_th = c->th, best_cache = c->cache;
    for (int twl = 6; twl <= 10; ++twl) {
        if (twl > 6 && (1 << twl) > 2 * max_nx) break;
        for (int th : {1, 2, 4, 8, 16}) {
            if (!tile_ok(twl, th)) continue;
            // policies with and without nontemporal stores (bit 0), and the FP16
            // sweeps with LDS-staged rows (bit 4) and with node pairs (bit 5)
            // where they apply
            for (int cache : {1, 3, 4, 5, 9, 12, 13, 15, 29, 31, 37, 45, 47, 69, 71, 77, 79}) {
                if ((cache & 16) && !(c->staged_ok && twl <= 8 && (th == 1 || th == 2 || th == 4))) continue;
                if ((cache & 32) && !(c->paired_ok && twl >= 7 && (((1 << twl) * th / kBlock) % 2) == 0)) continue;
                // two steps per launch: whole chunks only, in launch pairs
                const bool two = (cache & 64) != 0;
                if (two && !(tb_applies(c->cfg, twl, th) && steps % 4 == 0 && (c->gstep & 1) == 0)) continue;
                c->cache = cache;
                rc = glbm_set_option(c, GLBM_OPT_TILE_WIDTH, 1 << twl);
                if (!rc) rc = glbm_set_option(c, GLBM_OPT_TILE_ROWS, th);
                if (!rc) rc = glbm_set_option(c, GLBM_OPT_TIMING, 1);
                if (rc) return rc;
                rc = enter(c);
                if (rc) return rc;
                int k = 0;
                if (two) {
                    for (int j = 0; j < steps / 2 && rc == GLBM_OK; ++j, k += 2)
                        rc = sweep_once(c, (int)((c->gstep + j) & 1), true);
                } else {
                    for (; k < steps && rc == GLBM_OK; ++k) rc = sweep_once(c, (int)((c->gstep + k) & 1));
                }
                double ms = 0.0;
                int64_t nl = 0;
                if (!rc) rc = glbm_sweep_time(c, &ms, &nl);
                // the sweeps advanced every active instance; keep the counters exact
                for (int i = 0; i < c->n_inst; ++i)
                    if (c->active_h[i]) c->steps[i] += k;
                c->gstep += k;
                c->snap_valid = false;
                const int lrc = leave(c);
                if (!rc) rc = lrc;
                if (rc) return rc;
                if (ms < best) {
                    best = ms;
                    best_twl = twl;
                    best_th = th;
                    best_cache = cache;
                }
            }
        }
    }
    rc = glbm_set_option(c, GLBM_OPT_TIMING, old_timing ? 1 : 0);
    if (!rc) rc = glbm_set_option(c, GLBM_OPT_TILE_WIDTH, 1 << best_twl);
    if (!rc) rc = glbm_set_option(c, GLBM_OPT_TILE_ROWS, best_th);
    if (!rc) rc = glbm_set_option(c, GLBM_OPT_CACHE, best_cache);
    if (rc) return rc;
    if (chosen) {
        chosen[0] = 1 << best_twl;
        chosen[1] = best_th;
        chosen[2] = best_cache;
    }
    return GLBM_OK;
}

int glbm_destroy(glbm_ctx c)
{
    if (!c) return GLBM_OK;
    if (c->work) (void)hipStreamSynchronize(c->work);
    free_graph(c);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->own_pop && c->pop_base) (void)hipFree(c->pop_base);
    (void)hipFree(c->cls_d);
    (void)hipFree(c->inst_d);
    (void)hipFree(c->tiles_d);
    (void)hipFree(c->tab_d);
    (void)hipFree(c->snap_d);
    (void)hipFree(c->part_d);
    (void)hipFree(c->res_d);
    (void)hipFree(c->flux_d);
    (void)hipFree(c->active_d);
    (void)hipFree(c->dsteps_d);
    if (c->res_p) (void)hipHostFree(c->res_p);
    if (c->active_p) (void)hipHostFree(c->active_p);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->work) (void)hipStreamDestroy(c->work);
    delete c;
    return GLBM_OK;
}

int glbm_cnn_features(glbm_ctx c, int32_t inst, double log10_pressure_mpa, uint16_t* x)
{
    g_err.clear();
    if (!c || !x) return fail(GLBM_EINVAL, "null argument");
    if (inst < 0 || inst >= c->n_inst) return fail(GLBM_EINVAL, "instance %d out of range", inst);
    int rc = check_tables(c);
    if (rc) return rc;
    std::vector<float> tab((size_t)kClasses * 8, 0.f);
    for (int k = 0; k < kClasses; ++k) {
        float* t = &tab[(size_t)k * 8];
        const int phase = k == 0 ? 0 : (k < 128 ? 1 : (k < kWallClass ? 2 : -1));
        if (phase >= 0) t[phase] = 1.f;
        const double kk = c->k_h[inst][k];
        t[3] = k == kWallClass ? 0.f : (float)c->eps_h[inst][k];
        t[4] = k == kWallClass ? 0.f : (std::isfinite(kk) ? (float)std::log10(kk) : 3.f);
        t[5] = (float)log10_pressure_mpa;
    }
    rc = enter(c);
    if (rc) return rc;
    Joined joined(c);
    float* d = nullptr;
    HIPCHK(hipMalloc(&d, tab.size() * sizeof(float)));
    const InstDev& I = c->inst_h[inst];
    const long long n = (long long)I.nx * I.ny * I.nz;
    hipError_t e = hipMemcpyAsync(d, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice, c->work);
    if (e == hipSuccess) e = launch_cnn_features(c->cls_d + I.cls_off, n, d, x, c->work);
    hipError_t es = hipStreamSynchronize(c->work);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(GLBM_EDEVICE, "features: %s", hipGetErrorString(e));
    HIPCHK(es);
    return joined.done();
}

int glbm_cnn_targets(glbm_ctx c, int32_t inst, double rho_scale, double u_scale, float* target, uint8_t* mask)
{
    g_err.clear();
    if (!c || !target || !mask) return fail(GLBM_EINVAL, "null argument");
    if (inst < 0 || inst >= c->n_inst) return fail(GLBM_EINVAL, "instance %d out of range", inst);
    if (!(rho_scale > 0) || !(u_scale > 0)) return fail(GLBM_EINVAL, "scales must be > 0");
    int rc = check_tables(c);
    if (rc) return rc;
    rc = enter(c);
    if (rc) return rc;
    Joined joined(c);
    const InstDev& I = c->inst_h[inst];
    const long long n = (long long)I.nx * I.ny * I.nz;
    double* d = nullptr;
    HIPCHK(hipMalloc(&d, (size_t)4 * n * sizeof(double)));
    hipError_t e = launch_get_fields(c->cfg, c->args(c->gstep), inst, I.ntiles, d, d + n, nullptr, c->work);
    if (e == hipSuccess)
        e = launch_cnn_targets(d, d + n, c->cls_d + I.cls_off, n, rho_scale, u_scale, target, mask, c->work);
    hipError_t es = hipStreamSynchronize(c->work);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(GLBM_EDEVICE, "targets: %s", hipGetErrorString(e));
    HIPCHK(es);
    return joined.done();
}

int glbm_cnn_apply(glbm_ctx c, int32_t inst, const float* y, double rho_scale, double u_scale)
{
    g_err.clear();
    if (!c || !y) return fail(GLBM_EINVAL, "null argument");
    if (inst < 0 || inst >= c->n_inst) return fail(GLBM_EINVAL, "instance %d out of range", inst);
    int rc = check_tables(c);
    if (rc) return rc;
    rc = enter(c);
    if (rc) return rc;
    Joined joined(c);
    const InstDev& I = c->inst_h[inst];
    const long long n = (long long)I.nx * I.ny * I.nz;
    float* d = nullptr;
    HIPCHK(hipMalloc(&d, (size_t)4 * n * sizeof(float)));
    hipError_t e = launch_cnn_apply(y, n, rho_scale, u_scale, d, d + n, c->work);
    rc = e == hipSuccess ? set_fields_impl(c, inst, d, d + n, 0) : fail(GLBM_EDEVICE, "apply: %s", hipGetErrorString(e));
    hipError_t es = hipStreamSynchronize(c->work);
    (void)hipFree(d);
    if (rc) return rc;
    HIPCHK(es);
    return joined.done();
}

int glbm_cnn_apply_noalloc(glbm_ctx c, int32_t inst, const float* y, double rho_scale, double u_scale)
{
    g_err.clear();
    if (!c || !y) return fail(GLBM_EINVAL, "null argument");
    if (inst < 0 || inst >= c->n_inst) return fail(GLBM_EINVAL, "instance %d out of range", inst);
    const InstDev& I = c->inst_h[inst];
    const long long n = (long long)I.nx * I.ny * I.nz;
    if (n > GLBM_NOALLOC_MAX_NODES)
        return fail(GLBM_EINVAL, "instance %d has %lld nodes, more than the %d of the allocation-free scratch", inst, n,
                    (int)GLBM_NOALLOC_MAX_NODES);
    int rc = check_tables(c);
    if (rc) return rc;
    float* d = scratch_of(c->device);
    if (!d) return fail(GLBM_ESTATE, "no scratch address for device %d", c->device);
    rc = enter(c);
    if (rc) return rc;
    Joined joined(c);
    // every element of the 4n staged floats is written before it is read: nothing to clear
    const hipError_t e = launch_cnn_apply(y, n, rho_scale, u_scale, d, d + n, c->work);
    if (e != hipSuccess) return fail(GLBM_EDEVICE, "apply: %s", hipGetErrorString(e));
    rc = set_fields_impl(c, inst, d, d + n, 0);
    if (rc) return rc;
    return joined.done();
}

int glbm_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream)
{
    g_err.clear();
    if (!src || !dst) return fail(GLBM_EINVAL, "null pointer");
    if ((bytes & 15) || (reinterpret_cast<uintptr_t>(src) & 15) || (reinterpret_cast<uintptr_t>(dst) & 15))
        return fail(GLBM_EINVAL, "pointers and size must be multiples of 16 bytes");
    HIPCHK(launch_stream_copy(src, dst, bytes, static_cast<hipStream_t>(hip_stream)));
    return GLBM_OK;
}

int glbm_velocity_set(int32_t lattice, int32_t* e, double* w)
{
    g_err.clear();
    if (lattice == GLBM_D2Q9) {
        static const int v[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}, {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
        for (int i = 0; i < 9; ++i) {
            if (e) {
                e[3 * i] = v[i][0];
                e[3 * i + 1] = v[i][1];
                e[3 * i + 2] = 0;
            }
            if (w) w[i] = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        }
        return GLBM_OK;
    }
    if (lattice == GLBM_D3Q19) {
        static const int v[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                                     {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                     {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                     {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
        for (int i = 0; i < 19; ++i) {
            if (e)
                for (int a = 0; a < 3; ++a) e[3 * i + a] = v[i][a];
            if (w) w[i] = i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
        }
        return GLBM_OK;
    }
    return fail(GLBM_EINVAL, "lattice must be 9 or 19");
}

}  // extern "C"
