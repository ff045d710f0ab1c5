// libzeta3 entry points: argument validation, error reporting, orchestration.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <mutex>
#include <vector>

#include "z3_internal.h"

namespace z3 {

static thread_local char g_err[1024] = "";

z3_status fail(z3_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

z3_status check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return Z3_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        return fail(Z3_ERR_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e));
    }
    return fail(Z3_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

z3_status check_launch(const char *what) { return check_hip(hipGetLastError(), what); }

// Largest single device allocation the library makes (z3_set_device_alloc_limit; initial
// value from Z3_DEVICE_ALLOC_LIMIT_MB, else unlimited).  Checked before any device call, so a
// request above it fails with Z3_ERR_OUT_OF_MEMORY exactly as a failed allocation does.
static size_t initial_alloc_limit()
{
    if (const char *e = getenv("Z3_DEVICE_ALLOC_LIMIT_MB")) {
        char *end = nullptr;
        const double mb = strtod(e, &end);
        if (end != e && mb >= 0.0 && mb < 1e12) return (size_t)(mb * 1048576.0);
    }
    return SIZE_MAX;
}
static std::atomic<size_t> g_alloc_limit{initial_alloc_limit()};

z3_status alloc_allowed(size_t bytes, const char *what)
{
    const size_t lim = g_alloc_limit.load(std::memory_order_relaxed);
    if (bytes > lim)
        return fail(Z3_ERR_OUT_OF_MEMORY, "%s: %zu bytes exceed the device allocation limit of %zu bytes", what, bytes,
                    lim);
    return Z3_OK;
}

// One private memory pool per device, never trimmed: the fused estimator allocates its
// chunk workspace stream-ordered on every call, and the pool hands the same memory back
// without a device-wide synchronisation.
static std::mutex g_pool_mu;
static hipMemPool_t g_pools[64] = {};

static z3_status pool_for_current_device(hipMemPool_t *pool)
{
    int dev = 0;
    z3_status st = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st != Z3_OK) return st;
    if (dev < 0 || dev >= 64) return fail(Z3_ERR_UNSUPPORTED, "device ordinal %d", dev);
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!g_pools[dev]) {
        hipMemPoolProps props = {};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t p;
        if ((st = check_hip(hipMemPoolCreate(&p, &props), "hipMemPoolCreate")) != Z3_OK) return st;
        uint64_t keep = UINT64_MAX;
        if ((st = check_hip(hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep),
                            "hipMemPoolSetAttribute")) != Z3_OK)
            return st;
        g_pools[dev] = p;
    }
    *pool = g_pools[dev];
    return Z3_OK;
}

// Scratch blocks kept per device between calls.  A chunk workspace has the same size call
// after call; handing the same block back without returning it to the runtime avoids the
// re-mapping that stream-ordered pool allocations of ~16 GiB have cost now and then (0.2-1.3 s
// for one allocation, measured, with the pool's release threshold at its maximum).  When a
// call gives a block back, an event is recorded on its stream; a later call, on any stream,
// waits for that event before it uses the block (free on the same stream, whose order already
// implies it), so a block moves between streams as safely as pool memory does.  Within a call
// a block is busy until scratch_free.  Idle blocks too small for a new request are given back
// to the pool first.
struct WsBlock {
    int dev;
    void *p;
    size_t bytes;
    bool busy;
    hipEvent_t done;  // recorded when the block was last given back
};
static std::mutex g_ws_mu;
static std::vector<WsBlock> g_ws;

static thread_local CallScope *t_scope = nullptr;

CallScope::CallScope(z3_index i, hipStream_t s) : idx(i), prev(t_scope)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess) capturing = cs != hipStreamCaptureStatusNone;
    t_scope = this;
}

CallScope::~CallScope()
{
    if (idx && !capturing && used > idx->ws_peak) idx->ws_peak = used;
    t_scope = prev;
}

z3_status scratch_alloc(void **p, size_t bytes, hipStream_t s)
{
    *p = nullptr;
    const size_t aligned = ((bytes ? bytes : 1) + 255) / 256 * 256;
    CallScope *sc = t_scope;
    if (sc && sc->capturing) {
        z3_index idx = sc->idx;
        if (!idx) return fail(Z3_ERR_UNSUPPORTED, "this call needs scratch memory and cannot be captured in a graph");
        if (sc->used + aligned > idx->cap_bytes)
            return fail(Z3_ERR_INVALID_ARG,
                        "graph capture needs %zu bytes of index workspace, %zu reserved: run the same call once "
                        "eagerly, then z3_index_prepare_capture, before capturing",
                        sc->used + aligned, idx->cap_bytes);
        *p = static_cast<char *>(idx->cap_ws) + sc->used;
        sc->used += aligned;
        return Z3_OK;
    }
    z3_status st = alloc_allowed(aligned, "scratch workspace");
    if (st != Z3_OK) return st;
    int dev = 0;
    if ((st = check_hip(hipGetDevice(&dev), "hipGetDevice")) != Z3_OK) return st;
    std::vector<WsBlock> evict;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        WsBlock *best = nullptr;
        for (WsBlock &b : g_ws)
            if (!b.busy && b.dev == dev && b.bytes >= aligned && (!best || b.bytes < best->bytes)) best = &b;
        if (best) {
            if ((st = check_hip(hipStreamWaitEvent(s, best->done, 0), "hipStreamWaitEvent")) != Z3_OK) return st;
            best->busy = true;
            *p = best->p;
            if (sc) sc->used += aligned;
            return Z3_OK;
        }
        // no idle block fits: the device's idle blocks are all too small, give them back
        for (size_t i = 0; i < g_ws.size();) {
            if (!g_ws[i].busy && g_ws[i].dev == dev) {
                evict.push_back(g_ws[i]);
                g_ws[i] = g_ws.back();
                g_ws.pop_back();
            } else {
                ++i;
            }
        }
    }
    for (const WsBlock &b : evict) {
        // freed in the order of this stream, after the block's last use on its own
        (void)hipStreamWaitEvent(s, b.done, 0);
        (void)hipFreeAsync(b.p, s);
        (void)hipEventDestroy(b.done);
    }
    hipMemPool_t pool;
    if ((st = pool_for_current_device(&pool)) != Z3_OK) return st;
    hipEvent_t done = nullptr;
    if ((st = check_hip(hipEventCreateWithFlags(&done, hipEventDisableTiming), "hipEventCreateWithFlags")) != Z3_OK)
        return st;
    st = check_hip(hipMallocFromPoolAsync(p, aligned, pool, s), "hipMallocFromPoolAsync");
    if (st != Z3_OK) {
        (void)hipEventDestroy(done);
        return st;
    }
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        g_ws.push_back(WsBlock{dev, *p, aligned, true, done});
    }
    if (sc) sc->used += aligned;
    return Z3_OK;
}

void scratch_free(void *p, hipStream_t s)
{
    if (t_scope && t_scope->capturing) return;  // a slice of the index's capture workspace
    if (!p) return;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        for (WsBlock &b : g_ws)
            if (b.p == p) {
                // kept for the next call; its last use is this stream's work so far
                (void)hipEventRecord(b.done, s);
                b.busy = false;
                return;
            }
    }
    (void)hipFreeAsync(p, s);
}

// ---- kernel timing -------------------------------------------------------------------
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_events;
static int64_t g_prof_launches = 0;
static double g_prof_ms = 0.0;

static thread_local int t_prof_mute = 0;
ProfileMute::ProfileMute() { ++t_prof_mute; }
ProfileMute::~ProfileMute() { --t_prof_mute; }

bool profiling() { return g_prof_on; }

void profile_begin(hipStream_t s, hipEvent_t *ev0)
{
    *ev0 = nullptr;
    if (!g_prof_on || t_prof_mute > 0 || (t_scope && t_scope->capturing)) return;
    if (hipEventCreate(ev0) != hipSuccess) { *ev0 = nullptr; return; }
    (void)hipEventRecord(*ev0, s);
}

void profile_end(hipStream_t s, hipEvent_t ev0)
{
    if (!ev0) return;
    hipEvent_t ev1;
    if (hipEventCreate(&ev1) != hipSuccess) { (void)hipEventDestroy(ev0); return; }
    (void)hipEventRecord(ev1, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_events.emplace_back(ev0, ev1);
}

}  // namespace z3

using namespace z3;

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

Z3_API const char *z3_last_error(void) { return g_err; }

Z3_API const char *z3_status_string(z3_status s)
{
    switch (s) {
    case Z3_OK: return "ok";
    case Z3_ERR_INVALID_ARG: return "invalid argument";
    case Z3_ERR_OUT_OF_MEMORY: return "out of device memory";
    case Z3_ERR_HIP: return "HIP error";
    case Z3_ERR_UNSUPPORTED: return "unsupported";
    case Z3_ERR_OVERFLOW: return "overflow";
    }
    return "unknown status";
}

Z3_API z3_status z3_build_index(int64_t n, const double *xyz, const double *w, int nbins,
                                const double *edges_chord2, double cell_size, void *stream,
                                z3_index *out)
{
    if (!out) return fail(Z3_ERR_INVALID_ARG, "z3_build_index: out is NULL");
    *out = nullptr;
    if (n < 0) return fail(Z3_ERR_INVALID_ARG, "z3_build_index: n < 0");
    if (n >= ((int64_t)1 << 29)) return fail(Z3_ERR_OVERFLOW, "z3_build_index: n >= 2^29");
    if (n > 0 && !xyz) return fail(Z3_ERR_INVALID_ARG, "z3_build_index: xyz is NULL");
    if (nbins < 1 || nbins > Z3_MAX_NBINS)
        return fail(Z3_ERR_INVALID_ARG, "z3_build_index: nbins=%d outside 1..%d", nbins, Z3_MAX_NBINS);
    if (!edges_chord2) return fail(Z3_ERR_INVALID_ARG, "z3_build_index: edges_chord2 is NULL");
    for (int b = 0; b <= nbins; ++b)
        if (!std::isfinite(edges_chord2[b]))
            return fail(Z3_ERR_INVALID_ARG, "z3_build_index: edge %d is not finite", b);
    if (!(edges_chord2[0] > 0.0))
        return fail(Z3_ERR_INVALID_ARG, "z3_build_index: E_0 must be > 0 (excludes self-pairs)");
    for (int b = 0; b < nbins; ++b)
        if (!(edges_chord2[b + 1] > edges_chord2[b]))
            return fail(Z3_ERR_INVALID_ARG, "z3_build_index: edges not strictly increasing at %d", b);
    if (edges_chord2[nbins] > 4.0)
        return fail(Z3_ERR_INVALID_ARG, "z3_build_index: E_nbins > 4 (chord of antipodal points)");
    if (!std::isfinite(cell_size))
        return fail(Z3_ERR_INVALID_ARG, "z3_build_index: cell_size is not finite");
    return build_index_impl(n, xyz, w, nbins, edges_chord2, cell_size, as_stream(stream), out);
}

Z3_API z3_status z3_build_index_planar(int64_t n, const double *xy, const double *w, int nbins,
                                       const double *edges_d2, double cell_size, void *stream, z3_index *out)
{
    if (!out) return fail(Z3_ERR_INVALID_ARG, "z3_build_index_planar: out is NULL");
    *out = nullptr;
    if (n < 0) return fail(Z3_ERR_INVALID_ARG, "z3_build_index_planar: n < 0");
    if (n >= ((int64_t)1 << 29)) return fail(Z3_ERR_OVERFLOW, "z3_build_index_planar: n >= 2^29");
    if (n > 0 && !xy) return fail(Z3_ERR_INVALID_ARG, "z3_build_index_planar: xy is NULL");
    if (nbins < 1 || nbins > Z3_MAX_NBINS)
        return fail(Z3_ERR_INVALID_ARG, "z3_build_index_planar: nbins=%d outside 1..%d", nbins, Z3_MAX_NBINS);
    if (!edges_d2) return fail(Z3_ERR_INVALID_ARG, "z3_build_index_planar: edges_d2 is NULL");
    for (int b = 0; b <= nbins; ++b)
        if (!std::isfinite(edges_d2[b]))
            return fail(Z3_ERR_INVALID_ARG, "z3_build_index_planar: edge %d is not finite", b);
    if (!(edges_d2[0] > 0.0))
        return fail(Z3_ERR_INVALID_ARG, "z3_build_index_planar: E_0 must be > 0 (excludes self-pairs)");
    for (int b = 0; b < nbins; ++b)
        if (!(edges_d2[b + 1] > edges_d2[b]))
            return fail(Z3_ERR_INVALID_ARG, "z3_build_index_planar: edges not strictly increasing at %d", b);
    if (!std::isfinite(cell_size))
        return fail(Z3_ERR_INVALID_ARG, "z3_build_index_planar: cell_size is not finite");
    return build_index_impl(n, xy, w, nbins, edges_d2, cell_size, as_stream(stream), out, true);
}

Z3_API z3_status z3_index_set_values(z3_index idx, int nmaps, const double *x, void *stream)
{
    if (!idx) return fail(Z3_ERR_INVALID_ARG, "z3_index_set_values: idx is NULL");
    if (nmaps < 1) return fail(Z3_ERR_INVALID_ARG, "z3_index_set_values: nmaps < 1");
    if (idx->n > 0 && !x) return fail(Z3_ERR_INVALID_ARG, "z3_index_set_values: x is NULL");
    if ((double)nmaps * (double)idx->n >= 9.0e18 / 8.0)
        return fail(Z3_ERR_OVERFLOW, "z3_index_set_values: nmaps * n too large");
    return set_values_impl(idx, nmaps, x, as_stream(stream));
}

Z3_API z3_status z3_index_update_values(z3_index idx, const double *x, void *stream)
{
    if (!idx) return fail(Z3_ERR_INVALID_ARG, "z3_index_update_values: idx is NULL");
    if (idx->n > 0 && (idx->nmaps < 1 || !idx->d_v))
        return fail(Z3_ERR_INVALID_ARG, "z3_index_update_values: no values attached (z3_index_set_values)");
    if (idx->n > 0 && !x) return fail(Z3_ERR_INVALID_ARG, "z3_index_update_values: x is NULL");
    return update_values_impl(idx, x, as_stream(stream));
}

Z3_API z3_status z3_index_prepare_capture(z3_index idx, size_t min_bytes, size_t *reserved)
{
    if (!idx) return fail(Z3_ERR_INVALID_ARG, "z3_index_prepare_capture: idx is NULL");
    const size_t want = idx->ws_peak > min_bytes ? idx->ws_peak : min_bytes;
    if (want > idx->cap_bytes) {
        z3_status st = alloc_allowed(want, "z3_index_prepare_capture");
        if (st != Z3_OK) return st;
        st = check_hip(hipSetDevice(idx->device), "hipSetDevice");
        if (st == Z3_OK) st = check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize");
        if (st != Z3_OK) return st;
        void *ws = nullptr;
        if ((st = check_hip(hipMalloc(&ws, want), "hipMalloc (capture workspace)")) != Z3_OK) return st;
        // graphs captured against the previous workspace still point at it: keep it
        if (idx->cap_ws) idx->cap_retired.push_back(idx->cap_ws);
        idx->cap_ws = ws;
        idx->cap_bytes = want;
    }
    if (reserved) *reserved = idx->cap_bytes;
    return Z3_OK;
}

Z3_API z3_status z3_index_info(z3_index idx, int64_t *n, int *nbins, int *nmaps, int *nbands,
                               int64_t *ncells)
{
    if (!idx) return fail(Z3_ERR_INVALID_ARG, "z3_index_info: idx is NULL");
    if (n) *n = idx->n;
    if (nbins) *nbins = idx->nbins;
    if (nmaps) *nmaps = idx->nmaps;
    if (nbands) *nbands = idx->nbands;
    if (ncells) *ncells = idx->ncells;
    return Z3_OK;
}

__global__ void k_perm_to_i64(const int *perm, int64_t n, int64_t *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = perm[i];
}

Z3_API z3_status z3_index_perm(z3_index idx, int64_t *perm, void *stream)
{
    if (!idx) return fail(Z3_ERR_INVALID_ARG, "z3_index_perm: idx is NULL");
    if (idx->n == 0) return Z3_OK;
    if (!perm) return fail(Z3_ERR_INVALID_ARG, "z3_index_perm: perm is NULL");
    int64_t nb = (idx->n + 255) / 256;
    hipLaunchKernelGGL(k_perm_to_i64, dim3((unsigned)nb), dim3(256), 0, as_stream(stream),
                       idx->d_perm, idx->n, perm);
    return check_launch("k_perm_to_i64");
}

Z3_API void z3_index_free(z3_index idx)
{
    if (idx) free_index(idx);
}

static z3_status check_common(const char *fn, const z3_index_s *idx, int map, int m_max, int prec,
                              int64_t p0, int64_t p1)
{
    if (!idx) return fail(Z3_ERR_INVALID_ARG, "%s: idx is NULL", fn);
    if (m_max < 0 || m_max > Z3_MAX_MMAX)
        return fail(Z3_ERR_INVALID_ARG, "%s: m_max=%d outside 0..%d", fn, m_max, Z3_MAX_MMAX);
    if (prec != Z3_PREC_FP64 && prec != Z3_PREC_MIXED)
        return fail(Z3_ERR_INVALID_ARG, "%s: unknown precision %d", fn, prec);
    if (p0 < 0 || p1 < p0 || p1 > idx->n)
        return fail(Z3_ERR_INVALID_ARG, "%s: pivot range [%lld, %lld) outside [0, %lld]", fn,
                    (long long)p0, (long long)p1, (long long)idx->n);
    if (idx->n > 0 && (idx->nmaps < 1 || !idx->d_v))
        return fail(Z3_ERR_INVALID_ARG, "%s: no values attached (z3_index_set_values)", fn);
    if (idx->n > 0 && (map < 0 || map >= idx->nmaps))
        return fail(Z3_ERR_INVALID_ARG, "%s: map %d outside 0..%d", fn, map, idx->nmaps - 1);
    return Z3_OK;
}

Z3_API z3_status z3_accumulate_multipoles(z3_index idx, int map, int m_max, int prec, int norm,
                                          int64_t p0, int64_t p1, void *A, double *W,
                                          int64_t *counts, uint64_t *idhash, uint64_t *pair_total,
                                          void *stream)
{
    z3_status st = check_common("z3_accumulate_multipoles", idx, map, m_max, prec, p0, p1);
    if (st != Z3_OK) return st;
    if (norm != Z3_NORM_BIN && norm != Z3_NORM_NONE)
        return fail(Z3_ERR_INVALID_ARG, "z3_accumulate_multipoles: unknown norm %d", norm);
    if (p1 == p0) return Z3_OK;
    return launch_multipoles(idx, Pivots{idx->d_x, idx->d_y, idx->d_z}, map, m_max, prec, norm, p0, p1, A,
                             p1 - p0, W, counts, idhash, pair_total, as_stream(stream));
}

Z3_API z3_status z3_contract(int64_t npiv, int m_max, int nbins, int prec, const void *A,
                             const double *piv_v, double *zeta, void *stream)
{
    CallScope scope(nullptr, as_stream(stream));
    if (npiv < 0) return fail(Z3_ERR_INVALID_ARG, "z3_contract: npiv < 0");
    if (m_max < 0 || m_max > Z3_MAX_MMAX_HIST) return fail(Z3_ERR_INVALID_ARG, "z3_contract: bad m_max");
    if (nbins < 1 || nbins > Z3_MAX_NBINS) return fail(Z3_ERR_INVALID_ARG, "z3_contract: bad nbins");
    if (prec != Z3_PREC_FP64 && prec != Z3_PREC_MIXED)
        return fail(Z3_ERR_INVALID_ARG, "z3_contract: unknown precision %d", prec);
    if (!zeta) return fail(Z3_ERR_INVALID_ARG, "z3_contract: zeta is NULL");
    if (npiv == 0) return Z3_OK;
    if (!A || !piv_v) return fail(Z3_ERR_INVALID_ARG, "z3_contract: A or piv_v is NULL");
    size_t pb = contract_partial_bytes(npiv, m_max, nbins);
    void *part = nullptr;
    z3_status st = scratch_alloc(&part, pb, as_stream(stream));
    if (st != Z3_OK) return st;
    st = launch_contract(npiv, m_max, nbins, prec, A, npiv, piv_v, zeta, part, pb, as_stream(stream));
    scratch_free(part, as_stream(stream));
    return st;
}

static int64_t chunk_pivots(const z3_index_s *idx, int m_max, int prec)
{
    size_t elem = prec == Z3_PREC_FP64 ? 8 : 4;
    size_t per_piv = (size_t)(m_max + 1) * 2 * idx->nbins * elem;
    size_t budget = (size_t)16 << 30;
    if (const char *e = getenv("Z3_WORKSPACE_MB")) {
        long long mb = atoll(e);
        if (mb > 0) budget = (size_t)mb << 20;
    }
    int64_t c = (int64_t)(budget / per_piv);
    c = (c / kBlock) * kBlock;
    if (c < 16 * kBlock) c = 16 * kBlock;
    return c;
}

// Block shape of the MFMA many-map kernel (waves per block x 16-map tiles per wave).
// Unless the caller fixed it, the first eager call for an (m_max, precision) times every
// compiled shape on a 4096-pivot sample from the middle of the call's pivot range and
// keeps the fastest for the index.  All shapes give bit-identical results; a call made
// while its stream is being captured into a graph does not tune (it uses the tuned shape,
// else shape 0).
z3_status z3::batch_shape(z3_index idx, int m_max, int prec, int64_t p0, int64_t p1, hipStream_t s, int *out)
{
    if (idx->batch_shape_forced >= 0) {
        *out = idx->batch_shape_forced;
        return Z3_OK;
    }
    int &slot = idx->batch_shape_tuned[prec == Z3_PREC_MIXED ? 1 : 0][m_max];
    if (slot) {
        *out = slot - 1;
        return Z3_OK;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    z3_status st = check_hip(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
    if (st != Z3_OK) return st;
    if (cs != hipStreamCaptureStatusNone || p1 <= p0) {
        *out = 0;
        return Z3_OK;
    }
    const int64_t S = p1 - p0 < 4096 ? p1 - p0 : 4096;
    const int64_t q0 = p0 + (p1 - p0 - S) / 2;
    const size_t elem = prec == Z3_PREC_FP64 ? 8 : 4;
    const size_t stride = (size_t)S * (m_max + 1) * 2 * idx->nbins;
    void *wa = nullptr;  // pivot-major staging only: the transpose is the same for every shape
    if ((st = scratch_alloc(&wa, (size_t)idx->nmaps * stride * elem, s)) != Z3_OK) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    st = check_hip(hipEventCreate(&e0), "hipEventCreate");
    if (st == Z3_OK) st = check_hip(hipEventCreate(&e1), "hipEventCreate");
    float best_ms = 0.0f;
    int best = 0;
    for (int c = 0; c < batch_num_shapes() && st == Z3_OK; ++c) {
        // one untimed launch (code object load, caches), then one timed
        st = launch_multipoles_batch(idx, m_max, prec, c, q0, q0 + S, wa, nullptr, S, stride, nullptr, nullptr, s);
        if (st == Z3_OK) st = check_hip(hipEventRecord(e0, s), "hipEventRecord");
        if (st == Z3_OK) st = launch_multipoles_batch(idx, m_max, prec, c, q0, q0 + S, wa, nullptr, S, stride, nullptr, nullptr, s);
        if (st == Z3_OK) st = check_hip(hipEventRecord(e1, s), "hipEventRecord");
        if (st == Z3_OK) st = check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.0f;
        if (st == Z3_OK) st = check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        if (st == Z3_OK && (c == 0 || ms < best_ms)) {
            best_ms = ms;
            best = c;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    scratch_free(wa, s);
    if (st != Z3_OK) return st;
    slot = best + 1;
    *out = best;
    return Z3_OK;
}

Z3_API z3_status z3_index_set_batch_shape(z3_index idx, int waves, int maps_per_wave)
{
    if (!idx) return fail(Z3_ERR_INVALID_ARG, "z3_index_set_batch_shape: idx is NULL");
    if (waves == 0 && maps_per_wave == 0) {
        idx->batch_shape_forced = -1;
        return Z3_OK;
    }
    for (int c = 0; c < batch_num_shapes(); ++c) {
        int w, t;
        batch_shape_dims(c, &w, &t);
        if (w == waves && 16 * t == maps_per_wave) {
            idx->batch_shape_forced = c;
            return Z3_OK;
        }
    }
    return fail(Z3_ERR_INVALID_ARG, "z3_index_set_batch_shape: no compiled shape of %d waves x %d maps", waves,
                maps_per_wave);
}

Z3_API z3_status z3_index_batch_shape(z3_index idx, int m_max, int prec, int *waves, int *maps_per_wave)
{
    if (!idx || !waves || !maps_per_wave) return fail(Z3_ERR_INVALID_ARG, "z3_index_batch_shape: NULL argument");
    if (m_max < 0 || m_max > Z3_MAX_MMAX) return fail(Z3_ERR_INVALID_ARG, "z3_index_batch_shape: m_max=%d", m_max);
    if (prec != Z3_PREC_FP64 && prec != Z3_PREC_MIXED)
        return fail(Z3_ERR_INVALID_ARG, "z3_index_batch_shape: unknown precision %d", prec);
    const int c = idx->batch_shape_forced >= 0 ? idx->batch_shape_forced
                                                : idx->batch_shape_tuned[prec == Z3_PREC_MIXED ? 1 : 0][m_max] - 1;
    *waves = *maps_per_wave = 0;
    if (c >= 0) {
        int t;
        batch_shape_dims(c, waves, &t);
        *maps_per_wave = 16 * t;
    }
    return Z3_OK;
}

Z3_API z3_status z3_estimate(z3_index idx, int map, int m_max, int prec, int64_t p0, int64_t p1,
                             double *zeta, uint64_t *pair_total, void *stream)
{
    return z3_estimate_ex(idx, map, m_max, prec, 0u, p0, p1, zeta, pair_total, stream);
}

// The fused estimator's chunk loop.  Its workspace is either allocated per call
// (fixed == nullptr: the stream-ordered pool, or the index's capture workspace) or carved
// from a caller-held buffer of fixed_bytes, which then also bounds the chunk length.
static z3_status estimate_chunks(z3_index idx, int map, int m_max, int prec, bool no_self, int64_t p0, int64_t p1,
                                 double *zeta, uint64_t *pair_total, hipStream_t s, void *fixed, size_t fixed_bytes)
{
    z3_status st = Z3_OK;
    // Without the k = j terms the mixed path keeps FP64 storage and contraction: the exact
    // self terms removed from the diagonal can be most of |X_m(b)|^2, and the FP32 rounding
    // of X would leave an error relative to that full product, not to the smaller result.
    // Its multipoles are FP64 arithmetic on both paths, so this costs no time.
    if (no_self) prec = Z3_PREC_FP64;
    const size_t elem = prec == Z3_PREC_FP64 ? 8 : 4;
    const size_t per_piv = (size_t)(m_max + 1) * 2 * idx->nbins * elem;
    auto round256 = [](size_t b) { return (b + 255) / 256 * 256; };
    auto bytes_for = [&](int64_t c, size_t *ab, size_t *pb, size_t *sb) {
        *ab = (size_t)c * per_piv;
        *pb = contract_partial_bytes(c, m_max, idx->nbins);
        *sb = no_self ? (size_t)((c + kWave - 1) / kWave) * idx->nbins * sizeof(double) : 0;
        return round256(*ab) + round256(*pb) + round256(*sb);
    };
    int64_t chunk = chunk_pivots(idx, m_max, prec);
    if (chunk > p1 - p0) chunk = ((p1 - p0 + kBlock - 1) / kBlock) * kBlock;
    size_t abytes, pbytes, sbytes;
    if (fixed) {
        // the longest whole number of pivot blocks whose workspace fits the buffer
        int64_t c = (int64_t)(fixed_bytes / (per_piv + 64)) / kBlock * kBlock;
        if (c > chunk) c = chunk;
        while (c >= kBlock && bytes_for(c, &abytes, &pbytes, &sbytes) > fixed_bytes) c -= kBlock;
        if (c < kBlock)
            return fail(Z3_ERR_UNSUPPORTED, "z3_estimate_static: %d bins at m_max=%d need more than the %zu-byte static "
                        "workspace for %d pivots", idx->nbins, m_max, fixed_bytes, kBlock);
        chunk = c;
    }
    (void)bytes_for(chunk, &abytes, &pbytes, &sbytes);
    void *wa = nullptr, *wp = nullptr, *wsf = nullptr;
    if (fixed) {
        char *base = static_cast<char *>(fixed);
        wa = base;
        wp = base + round256(abytes);
        wsf = no_self ? base + round256(abytes) + round256(pbytes) : nullptr;
    } else {
        if ((st = scratch_alloc(&wa, abytes, s)) != Z3_OK) return st;
        st = scratch_alloc(&wp, pbytes, s);
        if (st == Z3_OK && no_self) st = scratch_alloc(&wsf, sbytes, s);
    }
    const double *v = idx->d_v + (size_t)map * idx->n;
    double *self_part = static_cast<double *>(wsf);
    for (int64_t c0 = p0; c0 < p1 && st == Z3_OK; c0 += chunk) {
        int64_t c1 = c0 + chunk < p1 ? c0 + chunk : p1;
        st = launch_multipoles(idx, Pivots{idx->d_x, idx->d_y, idx->d_z}, map, m_max, prec, Z3_NORM_BIN, c0, c1,
                               wa, c1 - c0, nullptr, nullptr, nullptr, pair_total, s, no_self ? v : nullptr,
                               self_part);
        if (st == Z3_OK)
            st = launch_contract(c1 - c0, m_max, idx->nbins, prec, wa, c1 - c0, v + c0, zeta, wp, pbytes, s);
        if (st == Z3_OK && no_self)
            st = launch_self_subtract(self_part, (c1 - c0 + kWave - 1) / kWave, m_max, idx->nbins, zeta, s);
    }
    if (!fixed) {
        scratch_free(wsf, s);
        scratch_free(wp, s);
        scratch_free(wa, s);
    }
    return st;
}

Z3_API z3_status z3_estimate_ex(z3_index idx, int map, int m_max, int prec, unsigned flags, int64_t p0,
                                int64_t p1, double *zeta, uint64_t *pair_total, void *stream)
{
    CallScope scope(idx, as_stream(stream));
    z3_status st = check_common("z3_estimate", idx, map, m_max, prec, p0, p1);
    if (st != Z3_OK) return st;
    if (!zeta) return fail(Z3_ERR_INVALID_ARG, "z3_estimate: zeta is NULL");
    if (flags & ~(unsigned)Z3_EST_EXCLUDE_SELF) return fail(Z3_ERR_INVALID_ARG, "z3_estimate_ex: unknown flags 0x%x", flags);
    if (p1 == p0) return Z3_OK;
    return estimate_chunks(idx, map, m_max, prec, (flags & Z3_EST_EXCLUDE_SELF) != 0, p0, p1, zeta, pair_total,
                           as_stream(stream), nullptr, 0);
}

// ---- angular-histogram estimator ---------------------------------------------------------

Z3_API z3_status z3_index_set_phi_bins(z3_index idx, int n_phi, const double *bounds)
{
    if (!idx) return fail(Z3_ERR_INVALID_ARG, "z3_index_set_phi_bins: idx is NULL");
    if (idx->planar) return fail(Z3_ERR_UNSUPPORTED, "z3_index_set_phi_bins: sky indexes only");
    if (n_phi < 4 || n_phi > Z3_MAX_NPHI)
        return fail(Z3_ERR_INVALID_ARG, "z3_index_set_phi_bins: n_phi=%d outside 4..%d", n_phi, Z3_MAX_NPHI);
    if (!bounds) return fail(Z3_ERR_INVALID_ARG, "z3_index_set_phi_bins: bounds is NULL");
    // the bin centres (k + 1/2) 2 pi / n_phi of the transform assume equal bins from north
    for (int k = 0; k < n_phi; ++k) {
        const double t = kTwoPi * k / n_phi;
        const double c = bounds[2 * k], sn = bounds[2 * k + 1];
        if (!(std::fabs(c - std::cos(t)) <= 1e-15 && std::fabs(sn - std::sin(t)) <= 1e-15))
            return fail(Z3_ERR_INVALID_ARG,
                        "z3_index_set_phi_bins: row %d is not (cos, sin)(2 pi %d / %d) to 1e-15", k, k, n_phi);
    }
    std::vector<double> tab(4 * (size_t)n_phi);
    for (int j = 0; j < 2 * n_phi; ++j) {
        tab[2 * j] = std::cos(kPi * j / n_phi);
        tab[2 * j + 1] = std::sin(kPi * j / n_phi);
    }
    z3_status st = alloc_allowed(2 * (size_t)n_phi * sizeof(double2), "z3_index_set_phi_bins");
    if (st == Z3_OK) st = check_hip(hipSetDevice(idx->device), "hipSetDevice");
    if (st != Z3_OK) return st;
    double2 *db = nullptr, *dt = nullptr;
    st = check_hip(hipMalloc((void **)&db, (size_t)n_phi * sizeof(double2)), "hipMalloc (angular bins)");
    if (st == Z3_OK) st = check_hip(hipMalloc((void **)&dt, 2 * (size_t)n_phi * sizeof(double2)), "hipMalloc (phases)");
    if (st == Z3_OK)
        st = check_hip(hipMemcpy(db, bounds, (size_t)n_phi * sizeof(double2), hipMemcpyHostToDevice), "copy bins");
    if (st == Z3_OK)
        st = check_hip(hipMemcpy(dt, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice), "copy phases");
    if (st == Z3_OK) st = check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (st != Z3_OK) {
        if (db) (void)hipFree(db);
        if (dt) (void)hipFree(dt);
        return st;
    }
    if (idx->d_phi_bounds) (void)hipFree(idx->d_phi_bounds);
    if (idx->d_phi_tab) (void)hipFree(idx->d_phi_tab);
    idx->d_phi_bounds = db;
    idx->d_phi_tab = dt;
    idx->n_phi = n_phi;
    return Z3_OK;
}

static z3_status check_hist(const char *fn, const z3_index_s *idx, int map, int m_max, int prec, int64_t p0,
                            int64_t p1)
{
    if (!idx) return fail(Z3_ERR_INVALID_ARG, "%s: idx is NULL", fn);
    if (idx->n_phi < 4) return fail(Z3_ERR_INVALID_ARG, "%s: no angular bins (z3_index_set_phi_bins)", fn);
    if (m_max < 0 || m_max > Z3_MAX_MMAX_HIST || 2 * m_max >= idx->n_phi)
        return fail(Z3_ERR_INVALID_ARG, "%s: m_max=%d outside 0..min(%d, n_phi/2 - 1) (n_phi=%d)", fn, m_max,
                    Z3_MAX_MMAX_HIST, idx->n_phi);
    // the remaining checks are those of the direct estimator (with any m_max <= Z3_MAX_MMAX)
    return check_common(fn, idx, map, 0, prec, p0, p1);
}

Z3_API z3_status z3_accumulate_histogram(z3_index idx, int map, int m_max, int prec, int norm, int64_t p0,
                                         int64_t p1, void *A, double *W, int64_t *counts, int *counts_phi,
                                         uint64_t *pair_total, void *stream)
{
    z3_status st = check_hist("z3_accumulate_histogram", idx, map, m_max, prec, p0, p1);
    if (st != Z3_OK) return st;
    if (norm != Z3_NORM_BIN && norm != Z3_NORM_NONE)
        return fail(Z3_ERR_INVALID_ARG, "z3_accumulate_histogram: unknown norm %d", norm);
    if (p1 == p0) return Z3_OK;
    return launch_multipoles_hist(idx, map, m_max, prec, norm, p0, p1, A, p1 - p0, W, counts, counts_phi,
                                  pair_total, as_stream(stream));
}

Z3_API z3_status z3_estimate_histogram(z3_index idx, int map, int m_max, int prec, int64_t p0, int64_t p1,
                                       double *zeta, uint64_t *pair_total, void *stream)
{
    CallScope scope(idx, as_stream(stream));
    z3_status st = check_hist("z3_estimate_histogram", idx, map, m_max, prec, p0, p1);
    if (st != Z3_OK) return st;
    if (!zeta) return fail(Z3_ERR_INVALID_ARG, "z3_estimate_histogram: zeta is NULL");
    if (p1 == p0) return Z3_OK;
    hipStream_t s = as_stream(stream);
    // Both precisions store the chunk's multipoles in FP64 and contract them in FP64: the
    // estimator's cost is the FP64 pair walk and transform, so FP32 storage would save
    // nothing measurable, and on fields whose zeta_m is a sum of terms of random sign it
    // would cost ~1e-6 at the higher multipoles this estimator is for.
    const int sprec = Z3_PREC_FP64;
    int64_t chunk = chunk_pivots(idx, m_max, sprec);
    if (chunk > p1 - p0) chunk = ((p1 - p0 + kBlock - 1) / kBlock) * kBlock;
    const size_t abytes = (size_t)chunk * (size_t)(m_max + 1) * 2 * idx->nbins * sizeof(double);
    const size_t pbytes = contract_partial_bytes(chunk, m_max, idx->nbins);
    void *wa = nullptr, *wp = nullptr;
    if ((st = scratch_alloc(&wa, abytes, s)) != Z3_OK) return st;
    st = scratch_alloc(&wp, pbytes, s);
    const double *v = idx->d_v + (size_t)map * idx->n;
    for (int64_t c0 = p0; c0 < p1 && st == Z3_OK; c0 += chunk) {
        const int64_t c1 = c0 + chunk < p1 ? c0 + chunk : p1;
        st = launch_multipoles_hist(idx, map, m_max, sprec, Z3_NORM_BIN, c0, c1, wa, c1 - c0, nullptr, nullptr,
                                    nullptr, pair_total, s);
        if (st == Z3_OK)
            st = launch_contract(c1 - c0, m_max, idx->nbins, sprec, wa, c1 - c0, v + c0, zeta, wp, pbytes, s);
    }
    scratch_free(wp, s);
    scratch_free(wa, s);
    return st;
}

// ---- the estimator without allocation ---------------------------------------------------
// Workspace of z3_estimate_static: a file-scope device array, one copy per GPU the library
// runs on, held until the process ends.  In host code its name is only a stand-in: the
// kernels get the address that hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes = (size_t)512 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64] = {};

static z3_status static_scratch(void **ptr)
{
    *ptr = nullptr;
    int dev = 0;
    z3_status st = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st != Z3_OK) return st;
    if (dev < 0 || dev >= 64) return fail(Z3_ERR_UNSUPPORTED, "device ordinal %d", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if ((st = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress (static workspace)")) !=
            Z3_OK)
            return st;
        if (!p) return fail(Z3_ERR_HIP, "hipGetSymbolAddress returned no address for the static workspace");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return Z3_OK;
}

Z3_API z3_status z3_estimate_static(z3_index idx, int map, int m_max, int prec, unsigned flags, int64_t p0,
                                    int64_t p1, double *zeta, uint64_t *pair_total, void *stream)
{
    z3_status st = check_common("z3_estimate_static", idx, map, m_max, prec, p0, p1);
    if (st != Z3_OK) return st;
    if (!zeta) return fail(Z3_ERR_INVALID_ARG, "z3_estimate_static: zeta is NULL");
    if (flags & ~(unsigned)Z3_EST_EXCLUDE_SELF)
        return fail(Z3_ERR_INVALID_ARG, "z3_estimate_static: unknown flags 0x%x", flags);
    if (p1 == p0) return Z3_OK;
    void *ws = nullptr;
    if ((st = static_scratch(&ws)) != Z3_OK) return st;
    ProfileMute mute;  // no timing events either
    return estimate_chunks(idx, map, m_max, prec, (flags & Z3_EST_EXCLUDE_SELF) != 0, p0, p1, zeta, pair_total,
                           as_stream(stream), ws, kStaticScratchBytes);
}

Z3_API z3_status z3_estimate_cross(z3_index idx, int map_a, int map_b, int map_c, int cyclic, int m_max,
                                   int prec, int64_t p0, int64_t p1, double *zeta, uint64_t *pair_total,
                                   void *stream)
{
    CallScope scope(idx, as_stream(stream));
    z3_status st = check_common("z3_estimate_cross", idx, map_a, m_max, prec, p0, p1);
    if (st == Z3_OK) st = check_common("z3_estimate_cross", idx, map_b, m_max, prec, p0, p1);
    if (st == Z3_OK) st = check_common("z3_estimate_cross", idx, map_c, m_max, prec, p0, p1);
    if (st != Z3_OK) return st;
    if (!zeta) return fail(Z3_ERR_INVALID_ARG, "z3_estimate_cross: zeta is NULL");
    if (cyclic != 0 && cyclic != 1) return fail(Z3_ERR_INVALID_ARG, "z3_estimate_cross: cyclic must be 0 or 1");
    if (p1 == p0) return Z3_OK;
    hipStream_t s = as_stream(stream);
    // the terms (pivot field; b1 field, b2 field) and the distinct fields whose multipoles they read
    const int fa[3] = {map_a, map_b, map_c};
    const int nterms = cyclic ? 3 : 1;
    int need[3], nneed = 0, slot_of[3];
    for (int t = 0; t < 3; ++t) {
        const int f = fa[t];
        if (!cyclic && t == 0) { slot_of[t] = -1; continue; }  // the single term reads B and C only
        int k = 0;
        while (k < nneed && need[k] != f) ++k;
        if (k == nneed) need[nneed++] = f;
        slot_of[t] = k;
    }
    // Three distinct fields of one group of kMapGroup attached maps (sky catalogues): one
    // pass of the register-tiled many-map kernel computes the group's multipoles with shared
    // pair geometry (Nside 2048, FP64: 15.1 s against 18.0 s for three one-map passes).  Both
    // precisions form the harmonics in FP64, so the choice is the same for both; two fields
    // run two one-map passes, as in z3_estimate_maps.
    const int grp = need[0] / kMapGroup;
    bool grouped = !idx->planar && idx->ngroups > grp && nneed > 2;
    for (int k = 0; k < nneed; ++k) grouped = grouped && need[k] / kMapGroup == grp;
    int top_slot = 0;  // the group kernel writes slots 0..top_slot at least
    if (grouped)
        for (int t = 0; t < 3; ++t) {
            slot_of[t] = fa[t] % kMapGroup;
            top_slot = slot_of[t] > top_slot ? slot_of[t] : top_slot;
        }
    const int nslots = grouped ? kMapGroup : nneed;
    int64_t chunk = chunk_pivots(idx, m_max, prec) / nslots;
    chunk = (chunk / kBlock) * kBlock;
    if (chunk < 16 * kBlock) chunk = 16 * kBlock;
    if (chunk > p1 - p0) chunk = ((p1 - p0 + kBlock - 1) / kBlock) * kBlock;
    const size_t elem = prec == Z3_PREC_FP64 ? 8 : 4;
    const size_t slot_elems = (size_t)chunk * (size_t)(m_max + 1) * 2 * idx->nbins;
    const size_t pbytes = cross_partial_bytes(chunk, m_max, idx->nbins);
    void *wa = nullptr, *wp = nullptr;
    if ((st = scratch_alloc(&wa, slot_elems * elem * nslots, s)) != Z3_OK) return st;
    st = scratch_alloc(&wp, pbytes, s);
    for (int64_t c0 = p0; c0 < p1 && st == Z3_OK; c0 += chunk) {
        const int64_t c1 = c0 + chunk < p1 ? c0 + chunk : p1;
        if (grouped)
            st = launch_multipoles_maps(idx, grp, top_slot + 1, m_max, prec, c0, c1, wa, c1 - c0, slot_elems, nullptr,
                                        pair_total, s);
        for (int k = 0; k < nneed && st == Z3_OK && !grouped; ++k)
            st = launch_multipoles(idx, Pivots{idx->d_x, idx->d_y, idx->d_z}, need[k], m_max, prec, Z3_NORM_BIN, c0,
                                   c1, static_cast<char *>(wa) + (size_t)k * slot_elems * elem, c1 - c0, nullptr,
                                   nullptr, nullptr, k == 0 ? pair_total : nullptr, s);
        for (int t = 0; t < nterms && st == Z3_OK; ++t) {
            // term t: pivot field fa[t], b1 field fa[t+1], b2 field fa[t+2] (cyclically)
            const int t1 = (t + 1) % 3, t2 = (t + 2) % 3;
            const void *X1 = static_cast<char *>(wa) + (size_t)slot_of[t1] * slot_elems * elem;
            const void *X2 = static_cast<char *>(wa) + (size_t)slot_of[t2] * slot_elems * elem;
            const double *v = idx->d_v + (size_t)fa[t] * idx->n + c0;
            st = launch_contract_cross(c1 - c0, m_max, idx->nbins, prec, X1, X2, c1 - c0, v, zeta, wp, pbytes, s);
        }
    }
    scratch_free(wp, s);
    scratch_free(wa, s);
    return st;
}

Z3_API z3_status z3_estimate_cross_catalogues(z3_index idx_b, int map_b, z3_index idx_c, int map_c, int64_t npiv,
                                              const double *piv_xyz, const double *piv_w, const double *piv_x,
                                              int m_max, int prec, int64_t p0, int64_t p1, double *zeta,
                                              uint64_t *pairs_b, uint64_t *pairs_c, double *sum_w, void *stream)
{
    CallScope scope(idx_b, as_stream(stream));
    if (!idx_b || !idx_c) return fail(Z3_ERR_INVALID_ARG, "z3_estimate_cross_catalogues: index is NULL");
    if (idx_b->planar != idx_c->planar)
        return fail(Z3_ERR_INVALID_ARG, "z3_estimate_cross_catalogues: one index on a plane, one on the sky");
    if (npiv < 0 || npiv >= (int64_t)0x7fffffff)
        return fail(Z3_ERR_INVALID_ARG, "z3_estimate_cross_catalogues: npiv=%lld", (long long)npiv);
    if (m_max < 0 || m_max > Z3_MAX_MMAX)
        return fail(Z3_ERR_INVALID_ARG, "z3_estimate_cross_catalogues: m_max=%d outside 0..%d", m_max, Z3_MAX_MMAX);
    if (prec != Z3_PREC_FP64 && prec != Z3_PREC_MIXED)
        return fail(Z3_ERR_INVALID_ARG, "z3_estimate_cross_catalogues: unknown precision %d", prec);
    if (p0 < 0 || p1 < p0 || p1 > npiv)
        return fail(Z3_ERR_INVALID_ARG, "z3_estimate_cross_catalogues: pivot range [%lld, %lld) outside [0, %lld]",
                    (long long)p0, (long long)p1, (long long)npiv);
    if (!zeta) return fail(Z3_ERR_INVALID_ARG, "z3_estimate_cross_catalogues: zeta is NULL");
    if (p1 > p0 && (!piv_xyz || !piv_x)) return fail(Z3_ERR_INVALID_ARG, "z3_estimate_cross_catalogues: NULL pivots");
    const z3_index_s *ix[2] = {idx_b, idx_c};
    const int mp[2] = {map_b, map_c};
    for (int k = 0; k < 2; ++k) {
        if (ix[k]->n > 0 && (ix[k]->nmaps < 1 || !ix[k]->d_v))
            return fail(Z3_ERR_INVALID_ARG, "z3_estimate_cross_catalogues: no values attached to index %d", k);
        if (ix[k]->n > 0 && (mp[k] < 0 || mp[k] >= ix[k]->nmaps))
            return fail(Z3_ERR_INVALID_ARG, "z3_estimate_cross_catalogues: map %d outside 0..%d", mp[k],
                        ix[k]->nmaps - 1);
    }
    if (idx_b->nbins != idx_c->nbins)
        return fail(Z3_ERR_INVALID_ARG, "z3_estimate_cross_catalogues: the indexes have different bins");
    for (int b = 0; b <= idx_b->nbins; ++b)
        if (idx_b->edges.e[b] != idx_c->edges.e[b])
            return fail(Z3_ERR_INVALID_ARG, "z3_estimate_cross_catalogues: the indexes have different bin edges");
    if (p1 == p0) return Z3_OK;
    hipStream_t s = as_stream(stream);
    z3_status st = Z3_OK;
    if (sum_w) {
        st = piv_w ? launch_weight_sum(piv_w + p0, p1 - p0, sum_w, s) : launch_add_scalar(sum_w, (double)(p1 - p0), s);
        if (st != Z3_OK) return st;
    }
    if (idx_b->n == 0 || idx_c->n == 0) return Z3_OK;  // an empty neighbour catalogue: every X is 0
    const int nb = idx_b->nbins;
    int64_t chunk = chunk_pivots(idx_b, m_max, prec) / 2;
    chunk = (chunk / kBlock) * kBlock;
    if (chunk < 16 * kBlock) chunk = 16 * kBlock;
    if (chunk > p1 - p0) chunk = ((p1 - p0 + kBlock - 1) / kBlock) * kBlock;
    const size_t elem = prec == Z3_PREC_FP64 ? 8 : 4;
    const size_t slot_bytes = (size_t)chunk * (size_t)(m_max + 1) * 2 * nb * elem;
    const size_t pbytes = cross_partial_bytes(chunk, m_max, nb);
    void *wa = nullptr, *wp = nullptr, *wz = nullptr, *wg = nullptr;
    if ((st = scratch_alloc(&wa, 2 * slot_bytes, s)) != Z3_OK) return st;
    st = scratch_alloc(&wp, pbytes, s);
    // plane: pivots are [2][npiv] (x, y); a zero row stands for z
    if (st == Z3_OK && idx_b->planar) st = scratch_alloc(&wz, (size_t)npiv * sizeof(double), s);
    if (st == Z3_OK && idx_b->planar) st = launch_fill(static_cast<double *>(wz), npiv, 0.0, s);
    // the pivots in catalogue B's band order (one sort), each chunk's gathered in that order
    const Pivots piv{piv_xyz, piv_xyz + npiv,
                     idx_b->planar ? static_cast<const double *>(wz) : piv_xyz + 2 * npiv};
    void *wperm = nullptr;
    if (st == Z3_OK) st = scratch_alloc(&wg, (size_t)4 * chunk * sizeof(double), s);
    if (st == Z3_OK) st = scratch_alloc(&wperm, (size_t)(p1 - p0) * sizeof(int), s);
    if (st == Z3_OK) st = sort_pivots(idx_b, piv, p0, p1 - p0, static_cast<int *>(wperm), s);
    double *gx = static_cast<double *>(wg), *gy = gx + chunk, *gz = gy + chunk, *gv = gz + chunk;
    for (int64_t c0 = p0; c0 < p1 && st == Z3_OK; c0 += chunk) {
        const int64_t c1 = c0 + chunk < p1 ? c0 + chunk : p1;
        const int64_t len = c1 - c0;
        st = gather_pivots(static_cast<const int *>(wperm) + (c0 - p0), len, piv, p0, piv_w, piv_x, gx, gy, gz, gv,
                           s);
        const Pivots sorted{gx, gy, gz};
        if (st == Z3_OK)
            st = launch_multipoles(idx_b, sorted, map_b, m_max, prec, Z3_NORM_BIN, 0, len, wa, len, nullptr, nullptr,
                                   nullptr, pairs_b, s);
        if (st == Z3_OK)
            st = launch_multipoles(idx_c, sorted, map_c, m_max, prec, Z3_NORM_BIN, 0, len,
                                   static_cast<char *>(wa) + slot_bytes, len, nullptr, nullptr, nullptr, pairs_c, s);
        if (st == Z3_OK)
            st = launch_contract_cross(len, m_max, nb, prec, wa, static_cast<char *>(wa) + slot_bytes, len, gv, zeta,
                                       wp, pbytes, s);
    }
    scratch_free(wperm, s);
    scratch_free(wg, s);
    scratch_free(wz, s);
    scratch_free(wp, s);
    scratch_free(wa, s);
    return st;
}

Z3_API z3_status z3_estimate_maps(z3_index idx, int m_max, int prec, int64_t p0, int64_t p1, double *zeta,
                                  uint64_t *pair_total, void *stream)
{
    CallScope scope(idx, as_stream(stream));
    z3_status st = check_common("z3_estimate_maps", idx, 0, m_max, prec, p0, p1);
    if (st != Z3_OK) return st;
    if (!zeta) return fail(Z3_ERR_INVALID_ARG, "z3_estimate_maps: zeta is NULL");
    if (p1 == p0) return Z3_OK;
    hipStream_t s = as_stream(stream);
    if (idx->nmaps == 1) return z3_estimate(idx, 0, m_max, prec, p0, p1, zeta, pair_total, stream);
    const size_t elem = prec == Z3_PREC_FP64 ? 8 : 4;
    const size_t per_map_piv = (size_t)(m_max + 1) * 2 * idx->nbins * elem;
    const size_t zstride = (size_t)(m_max + 1) * idx->nbins * idx->nbins * 2;
    // A group of four maps costs the register-tiled kernel the same however many of them are
    // real, about 2.5 one-map passes (Nside 512 and 2048, m_max = 10; both precisions form
    // the harmonics in FP64): one or two maps run as one-map passes, pairs counted once.  On
    // a plane (the many-map kernels take sky catalogues) every map runs a one-map pass.
    if (idx->nmaps <= 2 || idx->planar) {
        for (int k = 0; k < idx->nmaps && st == Z3_OK; ++k)
            st = z3_estimate(idx, k, m_max, prec, p0, p1, zeta + k * zstride, k == 0 ? pair_total : nullptr, stream);
        return st;
    }
    if (many_maps_on_mfma(idx, prec)) {
        // MFMA many-map kernel: all maps of a pivot chunk in one launch, then one
        // contraction launch for all maps
        int shape = 0;
        if ((st = batch_shape(idx, m_max, prec, p0, p1, s, &shape)) != Z3_OK) return st;
        // the contraction reads the kernel's pivot-major staging directly when its LDS tile
        // fits; otherwise the staging is transposed into the pivot-minor layout first
        const bool direct = gram_lds_fits(m_max, idx->nbins, prec);
        int64_t chunk = chunk_pivots(idx, m_max, prec) / ((direct ? 1 : 2) * idx->nmaps);
        chunk = (chunk / kBlock) * kBlock;
        if (chunk < 4 * kBlock) chunk = 4 * kBlock;
        if (chunk > p1 - p0) chunk = p1 - p0;
        const size_t pbytes = contract_partial_bytes(chunk, m_max, idx->nbins) * idx->nmaps;
        void *wa = nullptr, *wst = nullptr, *wp = nullptr;
        st = scratch_alloc(&wst, (size_t)idx->nmaps * chunk * per_map_piv, s);
        if (st == Z3_OK && !direct) st = scratch_alloc(&wa, (size_t)idx->nmaps * chunk * per_map_piv, s);
        if (st == Z3_OK) st = scratch_alloc(&wp, pbytes, s);
        for (int64_t c0 = p0; c0 < p1 && st == Z3_OK; c0 += chunk) {
            const int64_t c1 = c0 + chunk < p1 ? c0 + chunk : p1;
            const size_t stride = (size_t)(c1 - c0) * (m_max + 1) * 2 * idx->nbins;
            st = launch_multipoles_batch(idx, m_max, prec, shape, c0, c1, wst, wa, c1 - c0, stride, nullptr,
                                         pair_total, s);
            if (st != Z3_OK) break;
            if (direct)
                st = launch_contract_staged(c1 - c0, m_max, idx->nbins, prec, idx->nmaps, wst, idx->d_v + c0,
                                            (size_t)idx->n, zeta, zstride, wp, pbytes, s);
            else
                st = launch_contract_maps(c1 - c0, m_max, idx->nbins, prec, idx->nmaps, wa, c1 - c0, stride,
                                          idx->d_v + c0, (size_t)idx->n, zeta, zstride, wp, pbytes, s);
        }
        scratch_free(wp, s);
        scratch_free(wst, s);
        scratch_free(wa, s);
        return st;
    }
    int64_t chunk = chunk_pivots(idx, m_max, prec) / kMapGroup;
    chunk = (chunk / kBlock) * kBlock;
    if (chunk < 16 * kBlock) chunk = 16 * kBlock;
    if (chunk > p1 - p0) chunk = ((p1 - p0 + kBlock - 1) / kBlock) * kBlock;
    const size_t map_stride = (size_t)chunk * (m_max + 1) * 2 * idx->nbins;  // elements
    size_t pbytes = contract_partial_bytes(chunk, m_max, idx->nbins) * kMapGroup;
    void *wa = nullptr, *wp = nullptr;
    if ((st = scratch_alloc(&wa, (size_t)kMapGroup * chunk * per_map_piv, s)) != Z3_OK) return st;
    if ((st = scratch_alloc(&wp, pbytes, s)) != Z3_OK) {
        scratch_free(wa, s);
        return st;
    }
    // one or two maps left over after the full groups run one-map passes, which cost less than
    // a group pass (about 0.35 and 0.7 of one at Nside 512)
    const int rest = idx->nmaps % kMapGroup <= 2 ? idx->nmaps % kMapGroup : 0;
    const int ngroups = (idx->nmaps - rest + kMapGroup - 1) / kMapGroup;
    for (int g = 0; g < ngroups && st == Z3_OK; ++g) {
        for (int64_t c0 = p0; c0 < p1 && st == Z3_OK; c0 += chunk) {
            int64_t c1 = c0 + chunk < p1 ? c0 + chunk : p1;
            // the chunk's multipoles use a leading dimension equal to the chunk length
            const size_t stride = (size_t)(c1 - c0) * (m_max + 1) * 2 * idx->nbins;
            const int map0 = g * kMapGroup;
            const int nm = idx->nmaps - map0 < kMapGroup ? idx->nmaps - map0 : kMapGroup;
            st = launch_multipoles_maps(idx, g, nm, m_max, prec, c0, c1, wa, c1 - c0, stride, nullptr,
                                        g == 0 ? pair_total : nullptr, s);
            if (st == Z3_OK)
                st = launch_contract_maps(c1 - c0, m_max, idx->nbins, prec, nm, wa, c1 - c0, stride,
                                          idx->d_v + (size_t)map0 * idx->n + c0, (size_t)idx->n, zeta + map0 * zstride,
                                          zstride, wp, pbytes, s);
        }
    }
    (void)map_stride;
    scratch_free(wp, s);
    scratch_free(wa, s);
    for (int k = idx->nmaps - rest; k < idx->nmaps && st == Z3_OK; ++k)
        st = z3_estimate(idx, k, m_max, prec, p0, p1, zeta + k * zstride, nullptr, stream);
    return st;
}

Z3_API z3_status z3_estimate_pivots(z3_index idx, int map, int64_t npiv, const double *piv_xyz,
                                    const double *piv_w, const double *piv_x, int m_max, int prec,
                                    int64_t p0, int64_t p1, double *zeta, uint64_t *pair_total,
                                    double *sum_w, void *stream)
{
    CallScope scope(idx, as_stream(stream));
    if (!idx) return fail(Z3_ERR_INVALID_ARG, "z3_estimate_pivots: idx is NULL");
    if (npiv < 0) return fail(Z3_ERR_INVALID_ARG, "z3_estimate_pivots: npiv < 0");
    if (npiv >= (int64_t)0x7fffffff) return fail(Z3_ERR_OVERFLOW, "z3_estimate_pivots: npiv >= 2^31 - 1");
    if (m_max < 0 || m_max > Z3_MAX_MMAX)
        return fail(Z3_ERR_INVALID_ARG, "z3_estimate_pivots: m_max=%d outside 0..%d", m_max, Z3_MAX_MMAX);
    if (prec != Z3_PREC_FP64 && prec != Z3_PREC_MIXED)
        return fail(Z3_ERR_INVALID_ARG, "z3_estimate_pivots: unknown precision %d", prec);
    if (p0 < 0 || p1 < p0 || p1 > npiv)
        return fail(Z3_ERR_INVALID_ARG, "z3_estimate_pivots: pivot range [%lld, %lld) outside [0, %lld]",
                    (long long)p0, (long long)p1, (long long)npiv);
    if (!zeta) return fail(Z3_ERR_INVALID_ARG, "z3_estimate_pivots: zeta is NULL");
    if (p1 > p0 && (!piv_xyz || !piv_x)) return fail(Z3_ERR_INVALID_ARG, "z3_estimate_pivots: NULL pivots");
    if (idx->n > 0 && (idx->nmaps < 1 || !idx->d_v))
        return fail(Z3_ERR_INVALID_ARG, "z3_estimate_pivots: no values attached (z3_index_set_values)");
    if (idx->n > 0 && (map < 0 || map >= idx->nmaps))
        return fail(Z3_ERR_INVALID_ARG, "z3_estimate_pivots: map %d outside 0..%d", map, idx->nmaps - 1);
    if (p1 == p0) return Z3_OK;
    hipStream_t s = as_stream(stream);
    z3_status st = Z3_OK;
    if (sum_w) {
        st = piv_w ? launch_weight_sum(piv_w + p0, p1 - p0, sum_w, s) : launch_add_scalar(sum_w, (double)(p1 - p0), s);
        if (st != Z3_OK) return st;
    }
    if (idx->n == 0) return Z3_OK;  // no neighbours: no pairs, zeta unchanged
    int64_t chunk = chunk_pivots(idx, m_max, prec);
    if (chunk > p1 - p0) chunk = ((p1 - p0 + kBlock - 1) / kBlock) * kBlock;
    size_t elem = prec == Z3_PREC_FP64 ? 8 : 4;
    size_t abytes = (size_t)chunk * (size_t)(m_max + 1) * 2 * idx->nbins * elem;
    size_t pbytes = contract_partial_bytes(chunk, m_max, idx->nbins);
    void *wa = nullptr, *wp = nullptr, *wz = nullptr, *wg = nullptr;
    if ((st = scratch_alloc(&wa, abytes, s)) != Z3_OK) return st;
    st = scratch_alloc(&wp, pbytes, s);
    // plane: pivots are [2][npiv] (x, y); a zero row stands for z
    if (st == Z3_OK && idx->planar) st = scratch_alloc(&wz, (size_t)npiv * sizeof(double), s);
    if (st == Z3_OK && idx->planar) st = launch_fill(static_cast<double *>(wz), npiv, 0.0, s);
    // the pivots in the index's band order (one sort), each chunk's positions and values
    // gathered in that order
    const Pivots piv{piv_xyz, piv_xyz + npiv,
                     idx->planar ? static_cast<const double *>(wz) : piv_xyz + 2 * npiv};
    void *wperm = nullptr;
    if (st == Z3_OK) st = scratch_alloc(&wg, (size_t)4 * chunk * sizeof(double), s);
    if (st == Z3_OK) st = scratch_alloc(&wperm, (size_t)(p1 - p0) * sizeof(int), s);
    if (st == Z3_OK) st = sort_pivots(idx, piv, p0, p1 - p0, static_cast<int *>(wperm), s);
    double *gx = static_cast<double *>(wg), *gy = gx + chunk, *gz = gy + chunk, *gv = gz + chunk;
    for (int64_t c0 = p0; c0 < p1 && st == Z3_OK; c0 += chunk) {
        int64_t c1 = c0 + chunk < p1 ? c0 + chunk : p1;
        st = gather_pivots(static_cast<const int *>(wperm) + (c0 - p0), c1 - c0, piv, p0, piv_w, piv_x, gx, gy, gz,
                           gv, s);
        if (st == Z3_OK)
            st = launch_multipoles(idx, Pivots{gx, gy, gz}, map, m_max, prec, Z3_NORM_BIN, 0, c1 - c0, wa, c1 - c0,
                                   nullptr, nullptr, nullptr, pair_total, s);
        if (st == Z3_OK)
            st = launch_contract(c1 - c0, m_max, idx->nbins, prec, wa, c1 - c0, gv, zeta, wp, pbytes, s);
    }
    scratch_free(wperm, s);
    scratch_free(wg, s);
    scratch_free(wz, s);
    scratch_free(wp, s);
    scratch_free(wa, s);
    return st;
}

Z3_API z3_status z3_adjoint(z3_index idx, int map, int m_max, int64_t p0, int64_t p1, const double *G,
                            double scale, double *grad_x, void *stream)
{
    CallScope scope(idx, as_stream(stream));
    z3_status st = check_common("z3_adjoint", idx, map, m_max, Z3_PREC_FP64, p0, p1);
    if (st != Z3_OK) return st;
    if (!std::isfinite(scale)) return fail(Z3_ERR_INVALID_ARG, "z3_adjoint: scale is not finite");
    if (p1 == p0) return Z3_OK;
    if (!G || !grad_x) return fail(Z3_ERR_INVALID_ARG, "z3_adjoint: G or grad_x is NULL");
    return adjoint_impl(idx, map, m_max, p0, p1, G, scale, grad_x, as_stream(stream),
                        chunk_pivots(idx, m_max, Z3_PREC_FP64) / 2);
}

Z3_API z3_status z3_adjoint_maps(z3_index idx, int m_max, int64_t p0, int64_t p1, const double *G, double scale,
                                 double *grad_x, void *stream)
{
    CallScope scope(idx, as_stream(stream));
    z3_status st = check_common("z3_adjoint_maps", idx, 0, m_max, Z3_PREC_FP64, p0, p1);
    if (st != Z3_OK) return st;
    if (!std::isfinite(scale)) return fail(Z3_ERR_INVALID_ARG, "z3_adjoint_maps: scale is not finite");
    if (p1 == p0) return Z3_OK;
    if (!G || !grad_x) return fail(Z3_ERR_INVALID_ARG, "z3_adjoint_maps: G or grad_x is NULL");
    if (idx->nmaps == 1) return z3_adjoint(idx, 0, m_max, p0, p1, G, scale, grad_x, stream);
    if (idx->planar) {
        // plane: the many-map recompute kernels take sky catalogues, so one adjoint per map
        const size_t gstride = (size_t)(m_max + 1) * idx->nbins * idx->nbins * 2;
        for (int k = 0; k < idx->nmaps && st == Z3_OK; ++k)
            st = z3_adjoint(idx, k, m_max, p0, p1, G + k * gstride, scale, grad_x + (size_t)k * idx->n, stream);
        return st;
    }
    return adjoint_maps_impl(idx, m_max, p0, p1, G, scale, grad_x, as_stream(stream),
                             chunk_pivots(idx, m_max, Z3_PREC_FP64));
}

Z3_API z3_status z3_pivot_weight_sum(z3_index idx, int64_t p0, int64_t p1, double *out, void *stream)
{
    CallScope scope(idx, as_stream(stream));
    if (!idx) return fail(Z3_ERR_INVALID_ARG, "z3_pivot_weight_sum: idx is NULL");
    if (p0 < 0 || p1 < p0 || p1 > idx->n) return fail(Z3_ERR_INVALID_ARG, "z3_pivot_weight_sum: bad range");
    if (!out) return fail(Z3_ERR_INVALID_ARG, "z3_pivot_weight_sum: out is NULL");
    if (p1 == p0) return Z3_OK;
    return launch_weight_sum(idx->d_w + p0, p1 - p0, out, as_stream(stream));
}

Z3_API z3_status z3_finalize(int nmaps, int m_max, int nbins, double *zeta, const double *sum_w,
                             void *stream)
{
    if (nmaps < 1 || m_max < 0 || m_max > Z3_MAX_MMAX_HIST || nbins < 1 || nbins > Z3_MAX_NBINS)
        return fail(Z3_ERR_INVALID_ARG, "z3_finalize: bad sizes");
    if (!zeta || !sum_w) return fail(Z3_ERR_INVALID_ARG, "z3_finalize: NULL pointer");
    return launch_finalize(nmaps, m_max, nbins, zeta, sum_w, as_stream(stream));
}

Z3_API z3_status z3_resum(int m_max, int nbins, const double *zeta, int nphi, const double *phi,
                          double *out, void *stream)
{
    if (m_max < 0 || m_max > Z3_MAX_MMAX_HIST || nbins < 1 || nbins > Z3_MAX_NBINS || nphi < 0)
        return fail(Z3_ERR_INVALID_ARG, "z3_resum: bad sizes");
    if (nphi == 0) return Z3_OK;
    if (!zeta || !phi || !out) return fail(Z3_ERR_INVALID_ARG, "z3_resum: NULL pointer");
    return launch_resum(m_max, nbins, zeta, nphi, phi, out, as_stream(stream));
}

// Gamma-function poles of the k integral: at eta = 0 the arguments (1 + mt + a + n) / 2 and
// (1 - a - mt + n) / 2 are real; a non-positive integer there has no finite log Gamma.
static bool fftlog_pole(int n, int mt, double nu)
{
    const double a = 1.0 + nu;
    const double x[2] = {0.5 * (1.0 + mt + a + n), 0.5 * (1.0 - a - mt + n)};
    for (double v : x)
        if (v < 0.5 && std::fabs(v - std::nearbyint(v)) < 1e-9) return true;
    return false;
}

Z3_API z3_status z3_fftlog_workspace_size(int N, int nchi, int ntheta, int models_per_pass, size_t *bytes)
{
    if (!bytes) return fail(Z3_ERR_INVALID_ARG, "z3_fftlog_workspace_size: bytes is NULL");
    if (N < 4 || N > Z3_MAX_FFTLOG_N || N % 2 || nchi < 2 || ntheta < 1 || ntheta > Z3_MAX_FFTLOG_THETA ||
        models_per_pass < 1)
        return fail(Z3_ERR_INVALID_ARG, "z3_fftlog_workspace_size: bad sizes");
    *bytes = fftlog_workspace_bytes(N, nchi, ntheta, models_per_pass);
    return Z3_OK;
}

Z3_API z3_status z3_fftlog_a_functions(int N, const double *Pk, double k_min, double k_max, const double *nu,
                                       int nchi, double chi_min, double chi_max, int nmodels, const double *F,
                                       int ntheta, const double *theta, double *out, void *workspace,
                                       size_t workspace_bytes, void *stream)
{
    if (N < 4 || N > Z3_MAX_FFTLOG_N || N % 2 || nchi < 2 || ntheta < 1 || ntheta > Z3_MAX_FFTLOG_THETA ||
        nmodels < 0)
        return fail(Z3_ERR_INVALID_ARG, "z3_fftlog_a_functions: bad sizes");
    if (!nu) return fail(Z3_ERR_INVALID_ARG, "z3_fftlog_a_functions: nu is NULL");
    if (!(k_min > 0.0) || !(k_max > k_min) || !std::isfinite(k_max) || !(chi_min > 0.0) || !(chi_max > chi_min) ||
        !std::isfinite(chi_max))
        return fail(Z3_ERR_INVALID_ARG, "z3_fftlog_a_functions: need 0 < k_min < k_max and 0 < chi_min < chi_max");
    const int ns[4] = {0, 1, 1, 2}, mts[4] = {0, 1, -1, 0};
    for (int f = 0; f < 4; ++f) {
        if (!std::isfinite(nu[f]) || std::fabs(nu[f]) > 50.0)
            return fail(Z3_ERR_INVALID_ARG, "z3_fftlog_a_functions: nu[%d] = %g outside [-50, 50]", f, nu[f]);
        if (fftlog_pole(ns[f], mts[f], nu[f]))
            return fail(Z3_ERR_INVALID_ARG, "z3_fftlog_a_functions: nu[%d] = %g puts a Gamma pole on eta = 0", f,
                        nu[f]);
    }
    if (nmodels == 0) return Z3_OK;
    if (!Pk || !F || !theta || !out) return fail(Z3_ERR_INVALID_ARG, "z3_fftlog_a_functions: NULL pointer");
    const hipStream_t s = as_stream(stream);
    int chunk = nmodels < 65535 ? nmodels : 65535;  // one grid z index per model of a pass
    if (workspace) {
        if (reinterpret_cast<uintptr_t>(workspace) % 256)
            return fail(Z3_ERR_INVALID_ARG, "z3_fftlog_a_functions: workspace not 256-byte aligned");
        while (chunk > 1 && fftlog_workspace_bytes(N, nchi, ntheta, chunk) > workspace_bytes) chunk = (chunk + 1) / 2;
        if (fftlog_workspace_bytes(N, nchi, ntheta, chunk) > workspace_bytes)
            return fail(Z3_ERR_INVALID_ARG, "z3_fftlog_a_functions: workspace of %zu bytes holds no model (%zu needed)",
                        workspace_bytes, fftlog_workspace_bytes(N, nchi, ntheta, 1));
        return fftlog_impl(N, Pk, k_min, k_max, nu, nchi, chi_min, chi_max, nmodels, F, ntheta, theta, out,
                           workspace, chunk, s);
    }
    CallScope scope(nullptr, s);
    const size_t kMaxAuto = (size_t)1 << 30;
    while (chunk > 1 && fftlog_workspace_bytes(N, nchi, ntheta, chunk) > kMaxAuto) chunk = (chunk + 1) / 2;
    void *ws = nullptr;
    z3_status st = scratch_alloc(&ws, fftlog_workspace_bytes(N, nchi, ntheta, chunk), s);
    if (st != Z3_OK) return st;
    st = fftlog_impl(N, Pk, k_min, k_max, nu, nchi, chi_min, chi_max, nmodels, F, ntheta, theta, out, ws, chunk, s);
    scratch_free(ws, s);
    return st;
}

Z3_API z3_status z3_set_device_alloc_limit(size_t max_bytes)
{
    g_alloc_limit.store(max_bytes, std::memory_order_relaxed);
    return Z3_OK;
}

Z3_API z3_status z3_sync(void *stream)
{
    z3_status st = check_hip(hipStreamSynchronize(as_stream(stream)), "hipStreamSynchronize");
    if (st != Z3_OK) return st;
    return check_hip(hipGetLastError(), "asynchronous error");
}

Z3_API z3_status z3_profile_enable(int on)
{
    g_prof_on = on != 0;
    return Z3_OK;
}

Z3_API z3_status z3_profile_read(int64_t *launches, double *total_ms, int reset)
{
    std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        evs.swap(g_prof_events);
    }
    z3_status st = Z3_OK;
    for (auto &e : evs) {
        if (st == Z3_OK) st = check_hip(hipEventSynchronize(e.second), "hipEventSynchronize");
        float ms = 0.0f;
        if (st == Z3_OK) st = check_hip(hipEventElapsedTime(&ms, e.first, e.second), "hipEventElapsedTime");
        if (st == Z3_OK) {
            g_prof_ms += ms;
            g_prof_launches += 1;
        }
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    if (launches) *launches = g_prof_launches;
    if (total_ms) *total_ms = g_prof_ms;
    if (reset) {
        g_prof_launches = 0;
        g_prof_ms = 0.0;
    }
    return st;
}
