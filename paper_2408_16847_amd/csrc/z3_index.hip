// Sky-cell index: latitude bands x longitude cells, points sorted by cell.
//
// The paper finds the neighbours of each pivot with an octree (cBalls, "log N steps"
// per pivot).  On the GPU the catalogue is instead bucketed once into a regular grid:
// band k holds colatitudes [k H, (k+1) H), and inside band k the points are split into
// ncell_k equal longitude cells (one cell per point of the band on average).  Points are
// stored in cell order, so any longitude window of a band is a contiguous index range
// (two ranges when it wraps through phi = 0), which the multipole kernel streams with
// coalesced loads.  The order inside a cell is the original catalogue order, which makes
// the index and every later sum deterministic.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "z3_internal.h"

#ifndef Z3_BAND_HEIGHT_FACTOR
#define Z3_BAND_HEIGHT_FACTOR 1.4
#endif

namespace z3 {

// ---- small device helpers ------------------------------------------------------------

__device__ __forceinline__ void atomic_min_pos_double(double *addr, double v)
{
    // non-negative doubles order like their bit patterns
    atomicMin(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ void atomic_max_pos_double(double *addr, double v)
{
    atomicMax(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ double colatitude(double x, double y, double z)
{
    return atan2(sqrt(x * x + y * y), z);
}

__device__ __forceinline__ double longitude(double x, double y)
{
    double phi = atan2(y, x);
    if (phi < 0.0) phi += kTwoPi;
    return phi;
}

// ---- kernels ---------------------------------------------------------------------------

// Colatitude range of the positions and their largest deviation | |r|^2 - 1 | from unit
// length (non-finite -> +inf), one pass over the coordinates: a grid-stride extremum per
// thread, a block reduction, one atomic per block and quantity.
__global__ __launch_bounds__(256) void k_sky_range(const double *xyz, int64_t n, double *range /* [3] */)
{
    __shared__ double smin[256], smax[256], sdev[256];
    double lo = 4.0, hi = 0.0, dev = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
        const double th = colatitude(x, y, z);
        lo = fmin(lo, th);
        hi = fmax(hi, th);
        double d = fabs((x * x + y * y + z * z) - 1.0);
        if (!(d <= 1e300)) d = INFINITY;
        dev = fmax(dev, d);
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    sdev[threadIdx.x] = dev;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
            sdev[threadIdx.x] = fmax(sdev[threadIdx.x], sdev[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomic_min_pos_double(&range[0], smin[0]);
        atomic_max_pos_double(&range[1], smax[0]);
        if (sdev[0] > 0.0) atomic_max_pos_double(&range[2], sdev[0]);
    }
}

// colatitude ranges of the bands start empty: [lo0, 0]
__global__ void k_init_band_th(double *band_th, int nbands, double lo0)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nbands) return;
    band_th[2 * k] = lo0;
    band_th[2 * k + 1] = 0.0;
}

__global__ void k_set_int(int *p, int v) { *p = v; }

// Band of every point, with per-band counts and colatitude ranges.  Consecutive points
// usually share a band, so the lanes of a wave combine their updates per distinct band
// before touching global memory.
__global__ void k_band_of_point(const double *xyz, int64_t n, double inv_h, int nbands, int *band,
                                double *phi_out, int *band_count, double *band_th /* [nbands][2] */)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    int k = -1;
    double th = 0.0;
    if (valid) {
        const double x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
        th = colatitude(x, y, z);
        k = (int)(th * inv_h);
        k = k < 0 ? 0 : (k >= nbands ? nbands - 1 : k);
        band[i] = k;
        phi_out[i] = longitude(x, y);
    }
    const int lane = threadIdx.x & (kWave - 1);
    uint64_t todo = __ballot(valid);
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int kl = __shfl(k, leader, kWave);
        const bool mine = valid && k == kl;
        const uint64_t grp = __ballot(mine);
        double lo = mine ? th : 4.0, hi = mine ? th : 0.0;
        for (int o = 32; o > 0; o >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, o, kWave));
            hi = fmax(hi, __shfl_xor(hi, o, kWave));
        }
        if (lane == leader) {
            atomicAdd(&band_count[kl], (int)__popcll(grp));
            atomic_min_pos_double(&band_th[2 * kl], lo);
            atomic_max_pos_double(&band_th[2 * kl + 1], hi);
        }
        todo &= ~grp;
    }
}

__global__ void k_cell_of_point(int64_t n, const int *band, const double *phi, const Band *bands,
                                int *cell, int *cell_count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Band &bd = bands[band[i]];
    int c = (int)floor(phi[i] * ((double)bd.ncell / kTwoPi));
    c = c < 0 ? 0 : (c >= bd.ncell ? bd.ncell - 1 : c);
    int g = bd.cell_off + c;
    cell[i] = g;
    atomicAdd(&cell_count[g], 1);
}

// ---- pivots on a plane -------------------------------------------------------------------
// The plane reuses the sphere's grid: strips of y play the latitude bands and
// (x - x0) * sx in [0, 2 pi) the longitude of the cells.

// Per-block minima and maxima of x and y ([block][4]: min x, max x, min y, max y).
__global__ void k_plane_range(const double *xyz, int64_t n, double *part)
{
    __shared__ double sh[4][256];
    double v[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double x = xyz[i], y = xyz[n + i];
        v[0] = fmin(v[0], x); v[1] = fmax(v[1], x);
        v[2] = fmin(v[2], y); v[3] = fmax(v[3], y);
    }
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[0][threadIdx.x] = fmin(sh[0][threadIdx.x], sh[0][threadIdx.x + o]);
            sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + o]);
            sh[2][threadIdx.x] = fmin(sh[2][threadIdx.x], sh[2][threadIdx.x + o]);
            sh[3][threadIdx.x] = fmax(sh[3][threadIdx.x], sh[3][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// [2][n] plane positions -> [3][n] with z = 0 (the records and the d2 test then see
// dz = 0 exactly)
__global__ void k_plane_xyz(const double *xy, int64_t n, double *xyz)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    xyz[i] = xy[i];
    xyz[n + i] = xy[n + i];
    xyz[2 * n + i] = 0.0;
}

// Strip of every point (y - y0 in place of the colatitude) and its cell coordinate.
__global__ void k_band_of_point_plane(const double *xyz, int64_t n, double y0, double inv_h, double x0, double sx,
                                      int nbands, int *band, double *phi_out, int *band_count,
                                      double *band_th /* [nbands][2] */)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    int k = -1;
    double th = 0.0;
    if (valid) {
        th = xyz[n + i] - y0;  // >= 0: y0 is the smallest y
        k = (int)(th * inv_h);
        k = k < 0 ? 0 : (k >= nbands ? nbands - 1 : k);
        band[i] = k;
        phi_out[i] = (xyz[i] - x0) * sx;
    }
    const int lane = threadIdx.x & (kWave - 1);
    uint64_t todo = __ballot(valid);
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int kl = __shfl(k, leader, kWave);
        const bool mine = valid && k == kl;
        const uint64_t grp = __ballot(mine);
        double lo = mine ? th : INFINITY, hi = mine ? th : 0.0;
        for (int o = 32; o > 0; o >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, o, kWave));
            hi = fmax(hi, __shfl_xor(hi, o, kWave));
        }
        if (lane == leader) {
            atomicAdd(&band_count[kl], (int)__popcll(grp));
            atomic_min_pos_double(&band_th[2 * kl], lo);
            atomic_max_pos_double(&band_th[2 * kl + 1], hi);
        }
        todo &= ~grp;
    }
}

__global__ void k_scatter(int64_t n, const int *cell, const int *cell_start, int *cell_fill, int *order)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell[i];
    int pos = cell_start[c] + atomicAdd(&cell_fill[c], 1);
    order[pos] = (int)i;
}

// Put the points of every cell in increasing original index (cells hold ~1 point).
__global__ void k_sort_cells(int64_t ncells, const int *cell_start, int *order)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    int s = cell_start[c], e = cell_start[c + 1];
    for (int i = s + 1; i < e; ++i) {
        int v = order[i];
        int j = i - 1;
        while (j >= s && order[j] > v) {
            order[j + 1] = order[j];
            --j;
        }
        order[j + 1] = v;
    }
}

__global__ void k_gather_points(int64_t n, const int *perm, const double *xyz, const double *w,
                                double *x, double *y, double *z, double *ws)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    x[i] = xyz[j];
    y[i] = xyz[n + j];
    z[i] = xyz[2 * n + j];
    ws[i] = w ? w[j] : 1.0;
}

__global__ void k_gather_values(int64_t n, int nmaps, const int *perm, const double *wsorted,
                                const double *xv, double *v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    double w = wsorted[i];
    for (int m = 0; m < nmaps; ++m) v[(size_t)m * n + i] = w * xv[(size_t)m * n + j];
}

// Doubled-band layout: index-order point i of band k (first point s_k, n_k points) is
// stored at 2 s_k + (i - s_k) and again n_k positions later.
template <class T>
__global__ void k_double_bands(int64_t n, const int *band, const Band *bands, const T *in, T *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Band &bd = bands[band[i]];
    const int64_t q = 2 * (int64_t)bd.pt_start + (i - bd.pt_start);
    const T v = in[i];
    out[q] = v;
    out[q + bd.npts] = v;
}

__global__ void k_records(int64_t n, int nmaps, const int *band, const Band *bands, const double *x,
                          const double *y, const double *z, const double *v, double4 *rec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Band &bd = bands[band[i]];
    const int64_t q = 2 * (int64_t)bd.pt_start + (i - bd.pt_start);
    const double xi = x[i], yi = y[i], zi = z[i];
    for (int m = 0; m < nmaps; ++m) {
        const double4 r = make_double4(xi, yi, zi, v[(size_t)m * n + i]);
        rec[(size_t)m * 2 * n + q] = r;
        rec[(size_t)m * 2 * n + q + bd.npts] = r;
    }
}

// Values of map group g in doubled-band order, kMapGroup maps interleaved per point
// (missing maps of the last group are 0).
__global__ void k_group_values(int64_t n, int nmaps, const int *band, const Band *bands, const double *v,
                               double *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Band &bd = bands[band[i]];
    const int64_t q = 2 * (int64_t)bd.pt_start + (i - bd.pt_start);
    const int ng = (nmaps + kMapGroup - 1) / kMapGroup;
    for (int g = 0; g < ng; ++g) {
        double *o = out + (size_t)g * 2 * n * kMapGroup;
        for (int k = 0; k < kMapGroup; ++k) {
            const int m = g * kMapGroup + k;
            const double val = m < nmaps ? v[(size_t)m * n + i] : 0.0;
            o[(size_t)q * kMapGroup + k] = val;
            o[(size_t)(q + bd.npts) * kMapGroup + k] = val;
        }
    }
}

// Per-record value matrix of the MFMA many-map kernel: row q of the doubled-band order
// holds the ldv map values of its point (maps >= nmaps are 0).  One thread per (point, map).
__global__ void k_value_matrix(int64_t n, int nmaps, int ldv, const int *band, const Band *bands, const double *v,
                               double *out64, float *out32)
{
    const int64_t total = n * ldv;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / ldv;
        const int m = (int)(t - i * ldv);
        const Band &bd = bands[band[i]];
        const int64_t q = 2 * (int64_t)bd.pt_start + (i - bd.pt_start);
        const double val = m < nmaps ? v[(size_t)m * n + i] : 0.0;
        out64[q * ldv + m] = val;
        out64[(q + bd.npts) * ldv + m] = val;
        out32[q * ldv + m] = (float)val;
        out32[(q + bd.npts) * ldv + m] = (float)val;
    }
}

__global__ void k_gather_int(int64_t n, const int *perm, const int *in, int *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[perm[i]];
}

__global__ void k_fill_double(double *p, int64_t n, double v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_int(int *p, int64_t n, int v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---- exclusive scan of int counts (n < 2^31 total) -----------------------------------

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;

__global__ void k_scan_tiles(const int *in, int64_t n, int *out, int *tile_sums)
{
    __shared__ int sh[kScanThreads];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int v[kScanPer];
    int sum = 0;
    for (int k = 0; k < kScanPer; ++k) {
        int64_t i = base + k;
        v[k] = i < n ? in[i] : 0;
        sum += v[k];
    }
    sh[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int t = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int run = sh[threadIdx.x] - sum;  // exclusive prefix of this thread
    for (int k = 0; k < kScanPer; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
    if (threadIdx.x == kScanThreads - 1) tile_sums[blockIdx.x] = sh[threadIdx.x];
}

__global__ void k_scan_add(int *out, int64_t n, const int *tile_offsets)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_offsets[i / kScanTile];
}

// out[i] = sum_{k<i} in[k] for i in [0, n) (the caller stores the total in out[n]).
static z3_status exclusive_scan(const int *in, int64_t n, int *out, hipStream_t s)
{
    int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles < 1) tiles = 1;
    const size_t bytes = (size_t)(tiles + 1) * sizeof(int);
    // both partial-sum buffers are released (stream-ordered) on every path out
    struct Tmp {
        int *p = nullptr;
        hipStream_t s;
        ~Tmp() { if (p) (void)hipFreeAsync(p, s); }
    } sums{nullptr, s}, offs{nullptr, s};
    z3_status st = alloc_allowed(bytes, "scan alloc");
    if (st == Z3_OK) st = check_hip(hipMallocAsync((void **)&sums.p, bytes, s), "scan alloc");
    if (st != Z3_OK) return st;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, in, n, out, sums.p);
    if ((st = check_launch("k_scan_tiles")) != Z3_OK) return st;
    if (tiles > 1) {
        st = alloc_allowed(bytes, "scan alloc");
        if (st == Z3_OK) st = check_hip(hipMallocAsync((void **)&offs.p, bytes, s), "scan alloc");
        if (st != Z3_OK) return st;
        if ((st = exclusive_scan(sums.p, tiles, offs.p, s)) != Z3_OK) return st;
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, offs.p);
        if ((st = check_launch("k_scan_add")) != Z3_OK) return st;
    }
    return Z3_OK;
}

static void free_ptrs(z3_index idx)
{
    void *ps[] = {idx->d_edges, idx->d_bands, idx->d_cell_start, idx->d_x, idx->d_y, idx->d_z,
                  idx->d_w, idx->d_perm, idx->d_band, idx->d_wdbl, idx->d_permdbl, idx->d_v, idx->d_rec,
                  idx->d_vgrp, idx->d_vmat64, idx->d_vmat32, idx->cap_ws, idx->d_phi_bounds, idx->d_phi_tab};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    for (void *p : idx->cap_retired) (void)hipFree(p);
    idx->cap_retired.clear();
}

void free_index(z3_index idx)
{
    (void)hipSetDevice(idx->device);
    (void)hipDeviceSynchronize();
    free_ptrs(idx);
    delete idx;
}

template <class T>
static z3_status dalloc(T **p, size_t count, const char *what)
{
    *p = nullptr;
    const size_t bytes = (count ? count : 1) * sizeof(T);
    const z3_status st = alloc_allowed(bytes, what);
    if (st != Z3_OK) return st;
    return check_hip(hipMalloc((void **)p, bytes), what);
}

static inline unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

z3_status build_index_impl(int64_t n, const double *xyz, const double *w, int nbins,
                           const double *edges, double cell_size, hipStream_t s, z3_index *out, bool planar)
{
    z3_index idx = new (std::nothrow) z3_index_s();
    if (!idx) return fail(Z3_ERR_OUT_OF_MEMORY, "z3_build_index: host allocation failed");
    (void)hipGetDevice(&idx->device);
    idx->n = n;
    idx->nbins = nbins;
    idx->planar = planar;
    z3_status st = Z3_OK;
    auto bail = [&](z3_status code) {
        (void)hipStreamSynchronize(s);
        free_ptrs(idx);
        delete idx;
        return code;
    };
    // plane: the [2][n] positions become [3][n] with z = 0 (freed on return; every path
    // out of this function synchronises the stream first)
    struct TmpBuf {
        double *p = nullptr;
        ~TmpBuf() { if (p) (void)hipFree(p); }
    } xyz3;
    if (planar && n > 0) {
        if ((st = dalloc(&xyz3.p, 3 * (size_t)n, "alloc plane positions")) != Z3_OK) return bail(st);
        hipLaunchKernelGGL(k_plane_xyz, dim3(grid_for(n)), dim3(256), 0, s, xyz, n, xyz3.p);
        if ((st = check_launch("k_plane_xyz")) != Z3_OK) return bail(st);
        xyz = xyz3.p;
    }
    // plane: bounding box of the points (x0 = min x, y0 = min y, extents lx, ly)
    double lx = 0.0, ly = 0.0, scale = 0.0;
    if (planar && n > 0) {
        const int nblk = (int)std::min<int64_t>((n + 255) / 256, 1024);
        double *d_part = nullptr;
        if ((st = dalloc(&d_part, 4 * (size_t)nblk, "alloc plane range")) != Z3_OK) return bail(st);
        hipLaunchKernelGGL(k_plane_range, dim3(nblk), dim3(256), 0, s, xyz, n, d_part);
        st = check_launch("k_plane_range");
        std::vector<double> part(4 * (size_t)nblk);
        if (st == Z3_OK)
            st = check_hip(hipMemcpyAsync(part.data(), d_part, part.size() * sizeof(double), hipMemcpyDeviceToHost, s),
                           "copy plane range");
        if (st == Z3_OK) st = check_hip(hipStreamSynchronize(s), "sync");
        (void)hipFree(d_part);
        if (st != Z3_OK) return bail(st);
        double v[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
        for (int b = 0; b < nblk; ++b) {
            v[0] = std::min(v[0], part[4 * b]); v[1] = std::max(v[1], part[4 * b + 1]);
            v[2] = std::min(v[2], part[4 * b + 2]); v[3] = std::max(v[3], part[4 * b + 3]);
        }
        if (!(std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]) && std::isfinite(v[3])))
            return bail(fail(Z3_ERR_INVALID_ARG, "z3_build_index_planar: positions are not finite"));
        idx->plane_x0 = v[0];
        idx->plane_y0 = v[2];
        lx = v[1] - v[0];
        ly = v[3] - v[2];
        scale = std::max(std::max(std::fabs(v[0]), std::fabs(v[1])), std::max(std::fabs(v[2]), std::fabs(v[3])));
        // cell coordinate (x - x0) sx stays below 2 pi
        idx->plane_sx = kTwoPi / (lx * (1.0 + 1e-12) + 1e-300 + 1e-15 * scale);
    }
    for (int b = 0; b <= nbins; ++b) {
        double e = edges[b];
        idx->edges.e[b] = e;
        if (planar) {
            // plane: rad_out is the enlarged radius, hav_out / hav_in the enlarged / reduced
            // squared radii of the window search (membership is the exact d2 test); the
            // absolute guard covers the rounding of coordinates of size `scale`
            const double g = 1e-14 * scale, r = sqrt(e);
            idx->edges.rad_out[b] = r * (1.0 + 1e-9) + g;
            idx->edges.hav_out[b] = idx->edges.rad_out[b] * idx->edges.rad_out[b];
            const double rin = std::max(0.0, r * (1.0 - 1e-9) - g);
            idx->edges.hav_in[b] = rin * rin;
            continue;
        }
        // Rounding guards for the window search only (membership is decided by the exact
        // d2 test): the FP64 squared chord of two FP64 unit vectors differs from the
        // exact chord by far less than 1e-9 relative at the separations supported here.
        idx->edges.hav_out[b] = 0.25 * e * (1.0 + 1e-9) + 1e-16;
        idx->edges.hav_in[b] = 0.25 * e * (1.0 - 1e-9) - 1e-16;
        double r = 2.0 * asin(std::min(1.0, sqrt(e) / 2.0));
        idx->edges.rad_out[b] = r * (1.0 + 1e-9) + 1e-12;
    }
    if ((st = dalloc(&idx->d_edges, 1, "alloc edges")) != Z3_OK) return bail(st);
    if ((st = check_hip(hipMemcpyAsync(idx->d_edges, &idx->edges, sizeof(EdgeTab), hipMemcpyHostToDevice, s),
                        "copy edges")) != Z3_OK)
        return bail(st);

    // ---- band height; sky positions: colatitude range and unit-length check --------------
    // Sky positions must be unit vectors: the windows are angular while membership is the
    // chord test on the raw vectors, and the windows' guards (1e-9 relative) cover a
    // deviation | |r|^2 - 1 | of up to kMaxNormDev only.
    double h = cell_size;
    double *d_range = nullptr;
    if ((st = dalloc(&d_range, 3, "alloc range")) != Z3_OK) return bail(st);
    if (planar && h <= 0.0) {
        // the same 1.4 x mean spacing as on the sphere
        double area = lx * ly;
        if (!(area > 0.0)) area = std::max(lx, ly) * std::max(lx, ly) / (double)std::max<int64_t>(n, 1);
        if (!(area > 0.0)) area = 1.0;
        h = Z3_BAND_HEIGHT_FACTOR * sqrt(area / (double)std::max<int64_t>(n, 1));
    } else if (!planar) {
        double rg[3] = {kPi, 0.0, 0.0};
        st = check_hip(hipMemcpyAsync(d_range, rg, sizeof(rg), hipMemcpyHostToDevice, s), "copy range");
        if (st == Z3_OK && n > 0) {
            unsigned g = grid_for(n) < 2048u ? grid_for(n) : 2048u;
            hipLaunchKernelGGL(k_sky_range, dim3(g), dim3(256), 0, s, xyz, n, d_range);
            st = check_launch("k_sky_range");
        }
        if (st == Z3_OK) st = check_hip(hipMemcpyAsync(rg, d_range, sizeof(rg), hipMemcpyDeviceToHost, s), "copy range");
        if (st == Z3_OK) st = check_hip(hipStreamSynchronize(s), "sync");
        if (st != Z3_OK) { (void)hipFree(d_range); return bail(st); }
        if (!(rg[2] <= kMaxNormDev)) {
            (void)hipFree(d_range);
            return bail(fail(Z3_ERR_INVALID_ARG,
                             "z3_build_index: positions are not unit vectors (max | |r|^2 - 1 | = %g, limit %g)", rg[2],
                             kMaxNormDev));
        }
        if (h <= 0.0) {
            double area = 2.0 * kPi * (cos(std::min(rg[0], rg[1])) - cos(std::max(rg[0], rg[1])));
            if (!(area > 0.0)) area = 1e-12;
            // 1.4 x the mean point spacing: about two HEALPix rings per band (ring spacing
            // 2 / (3 Nside) rad at low latitudes, mean spacing ~1.023 / Nside).  Each band
            // costs every pivot one longitude window per bin, whose set-up (window bounds,
            // cell lookups, the mixed path's flush into FP64) outweighs the few candidates
            // that a taller band adds at the window ends; measured on HEALPix maps at Nside
            // 512 and 2048 against 0.6 (one ring per band) to 2.6, 1.3-1.8 is best.
            h = Z3_BAND_HEIGHT_FACTOR * sqrt(area / (double)std::max<int64_t>(n, 1));
        }
    }
    (void)hipFree(d_range);
    int nbands = 1;
    if (planar) {
        const double nb_d = std::floor(ly / h) + 1.0;
        if (!(nb_d <= (double)(1 << 26))) return bail(fail(Z3_ERR_INVALID_ARG, "z3_build_index_planar: cell_size too small"));
        nbands = (int)nb_d;
    } else {
        h = std::min(h, kPi);
        nbands = (int)std::ceil(kPi / h);
        if (nbands < 1) nbands = 1;
        if (nbands > (1 << 26)) return bail(fail(Z3_ERR_INVALID_ARG, "z3_build_index: cell_size too small"));
    }
    idx->band_h = h;
    idx->nbands = nbands;

    // ---- bands -------------------------------------------------------------------------
    int *d_band = nullptr, *d_band_count = nullptr, *d_cell = nullptr, *d_cell_count = nullptr;
    double *d_phi = nullptr, *d_band_th = nullptr;
    auto cleanup_tmp = [&]() {
        void *ps[] = {d_band, d_band_count, d_cell, d_cell_count, d_phi, d_band_th};
        for (void *p : ps)
            if (p) (void)hipFree(p);
    };
    auto bail2 = [&](z3_status code) {
        (void)hipStreamSynchronize(s);
        cleanup_tmp();
        return bail(code);
    };
    if ((st = dalloc(&d_band, n, "alloc band")) != Z3_OK) return bail2(st);
    if ((st = dalloc(&d_phi, n, "alloc phi")) != Z3_OK) return bail2(st);
    if ((st = dalloc(&d_band_count, nbands, "alloc band count")) != Z3_OK) return bail2(st);
    if ((st = dalloc(&d_band_th, 2 * (size_t)nbands, "alloc band theta")) != Z3_OK) return bail2(st);
    hipLaunchKernelGGL(k_fill_int, dim3(grid_for(nbands)), dim3(256), 0, s, d_band_count, (int64_t)nbands, 0);
    // th_lo starts at +big, th_hi at 0
    hipLaunchKernelGGL(k_init_band_th, dim3((unsigned)((nbands + 255) / 256)), dim3(256), 0, s, d_band_th, nbands,
                       planar ? INFINITY : 4.0);
    if ((st = check_launch("k_init_band_th")) != Z3_OK) return bail2(st);
    if (n > 0 && planar) {
        hipLaunchKernelGGL(k_band_of_point_plane, dim3(grid_for(n)), dim3(256), 0, s, xyz, n, idx->plane_y0, 1.0 / h,
                           idx->plane_x0, idx->plane_sx, nbands, d_band, d_phi, d_band_count, d_band_th);
        if ((st = check_launch("k_band_of_point_plane")) != Z3_OK) return bail2(st);
    } else if (n > 0) {
        hipLaunchKernelGGL(k_band_of_point, dim3(grid_for(n)), dim3(256), 0, s, xyz, n, 1.0 / h, nbands, d_band,
                           d_phi, d_band_count, d_band_th);
        if ((st = check_launch("k_band_of_point")) != Z3_OK) return bail2(st);
    }
    std::vector<int> bcount(nbands);
    std::vector<double> bth(2 * (size_t)nbands);
    st = check_hip(hipMemcpyAsync(bcount.data(), d_band_count, nbands * sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    if (st == Z3_OK)
        st = check_hip(hipMemcpyAsync(bth.data(), d_band_th, bth.size() * sizeof(double), hipMemcpyDeviceToHost, s), "copy");
    if (st == Z3_OK) st = check_hip(hipStreamSynchronize(s), "sync");
    if (st != Z3_OK) return bail2(st);

    // the multipole kernel addresses a band's doubled records (64 B per point) with 32-bit
    // byte offsets
    for (int k = 0; k < nbands; ++k)
        if ((int64_t)bcount[k] * 64 > (int64_t)UINT32_MAX)
            return bail2(fail(Z3_ERR_UNSUPPORTED, "z3_build_index: %d points in one latitude band", bcount[k]));
    std::vector<Band> bands(nbands);
    int64_t pt = 0, cells = 0;
    for (int k = 0; k < nbands; ++k) {
        Band &b = bands[k];
        std::memset(&b, 0, sizeof(Band));
        b.npts = bcount[k];
        b.pt_start = (int)pt;
        b.ncell = (int)std::max<int64_t>(1, (int64_t)kCellsPerPoint * b.npts);
        b.cell_off = (int)cells;
        b.cells_per_rad = (float)((double)b.ncell / kTwoPi);
        double lo = b.npts ? bth[2 * k] : k * h, hi = b.npts ? bth[2 * k + 1] : k * h;
        b.th_lo = lo;
        b.th_hi = hi;
        b.sh_lo = sin(0.5 * lo); b.ch_lo = cos(0.5 * lo);
        b.sh_hi = sin(0.5 * hi); b.ch_hi = cos(0.5 * hi);
        double slo = sin(lo), shi = sin(hi);
        double smin = std::min(slo, shi);
        double smax = (lo <= 0.5 * kPi && hi >= 0.5 * kPi) ? 1.0 : std::max(slo, shi);
        b.inv_smin = smin > 0.0 ? (float)(1.0 / smin) : INFINITY;
        b.inv_smax = smax > 0.0 ? (float)(1.0 / smax) : INFINITY;
        pt += b.npts;
        cells += b.ncell;
    }
    if (cells >= (int64_t)0x7fffffff || 2 * n >= (int64_t)0x7fffffff)
        return bail2(fail(Z3_ERR_OVERFLOW, "z3_build_index: too many points or cells"));
    idx->ncells = cells;
    if ((st = dalloc(&idx->d_bands, nbands, "alloc bands")) != Z3_OK) return bail2(st);
    st = check_hip(hipMemcpyAsync(idx->d_bands, bands.data(), nbands * sizeof(Band), hipMemcpyHostToDevice, s),
                   "copy bands");
    if (st != Z3_OK) return bail2(st);

    // ---- cells, sort -----------------------------------------------------------------------
    if ((st = dalloc(&d_cell, n, "alloc cell")) != Z3_OK) return bail2(st);
    if ((st = dalloc(&d_cell_count, cells + 1, "alloc cell count")) != Z3_OK) return bail2(st);
    if ((st = dalloc(&idx->d_cell_start, cells + 1, "alloc cell start")) != Z3_OK) return bail2(st);
    hipLaunchKernelGGL(k_fill_int, dim3(grid_for(cells + 1)), dim3(256), 0, s, d_cell_count, cells + 1, 0);
    if (n > 0) {
        hipLaunchKernelGGL(k_cell_of_point, dim3(grid_for(n)), dim3(256), 0, s, n, d_band, d_phi, idx->d_bands,
                           d_cell, d_cell_count);
        if ((st = check_launch("k_cell_of_point")) != Z3_OK) return bail2(st);
    }
    if ((st = exclusive_scan(d_cell_count, cells, idx->d_cell_start, s)) != Z3_OK) return bail2(st);
    // cell_start[cells] = n (bands are contiguous and cover all points)
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, idx->d_cell_start + cells, (int)n);
    if ((st = check_launch("k_set_int")) != Z3_OK) return bail2(st);
    if ((st = dalloc(&idx->d_perm, n, "alloc perm")) != Z3_OK) return bail2(st);
    hipLaunchKernelGGL(k_fill_int, dim3(grid_for(cells + 1)), dim3(256), 0, s, d_cell_count, cells + 1, 0);
    if (n > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(grid_for(n)), dim3(256), 0, s, n, d_cell, idx->d_cell_start,
                           d_cell_count, idx->d_perm);
        hipLaunchKernelGGL(k_sort_cells, dim3(grid_for(cells)), dim3(256), 0, s, cells, idx->d_cell_start,
                           idx->d_perm);
        if ((st = check_launch("k_scatter/k_sort_cells")) != Z3_OK) return bail2(st);
    }
    if ((st = dalloc(&idx->d_x, n, "alloc x")) != Z3_OK) return bail2(st);
    if ((st = dalloc(&idx->d_y, n, "alloc y")) != Z3_OK) return bail2(st);
    if ((st = dalloc(&idx->d_z, n, "alloc z")) != Z3_OK) return bail2(st);
    if ((st = dalloc(&idx->d_w, n, "alloc w")) != Z3_OK) return bail2(st);
    idx->unit_w = (w == nullptr);
    if ((st = dalloc(&idx->d_band, n, "alloc band")) != Z3_OK) return bail2(st);
    if ((st = dalloc(&idx->d_permdbl, 2 * n, "alloc perm2")) != Z3_OK) return bail2(st);
    if (!idx->unit_w && (st = dalloc(&idx->d_wdbl, 2 * n, "alloc w2")) != Z3_OK) return bail2(st);
    if (n > 0) {
        hipLaunchKernelGGL(k_gather_points, dim3(grid_for(n)), dim3(256), 0, s, n, idx->d_perm, xyz, w, idx->d_x,
                           idx->d_y, idx->d_z, idx->d_w);
        hipLaunchKernelGGL(k_gather_int, dim3(grid_for(n)), dim3(256), 0, s, n, idx->d_perm, d_band, idx->d_band);
        hipLaunchKernelGGL(k_double_bands<int>, dim3(grid_for(n)), dim3(256), 0, s, n, idx->d_band, idx->d_bands,
                           idx->d_perm, idx->d_permdbl);
        if (!idx->unit_w)
            hipLaunchKernelGGL(k_double_bands<double>, dim3(grid_for(n)), dim3(256), 0, s, n, idx->d_band,
                               idx->d_bands, idx->d_w, idx->d_wdbl);
        if ((st = check_launch("k_gather_points")) != Z3_OK) return bail2(st);
    }
    st = check_hip(hipStreamSynchronize(s), "sync");
    cleanup_tmp();
    if (st != Z3_OK) return bail(st);
    *out = idx;
    return Z3_OK;
}

// Rebuild every per-map array from new values x [nmaps][n] (catalogue order) into the
// buffers already attached: kernels only, on `s`.
static z3_status fill_values(z3_index idx, int nmaps, const double *x, hipStream_t s)
{
    z3_status st;
    if (idx->n == 0) return Z3_OK;
    hipLaunchKernelGGL(k_gather_values, dim3(grid_for(idx->n)), dim3(256), 0, s, idx->n, nmaps, idx->d_perm,
                       idx->d_w, x, idx->d_v);
    hipLaunchKernelGGL(k_records, dim3(grid_for(idx->n)), dim3(256), 0, s, idx->n, nmaps, idx->d_band,
                       idx->d_bands, idx->d_x, idx->d_y, idx->d_z, idx->d_v, idx->d_rec);
    if ((st = check_launch("k_gather_values/k_records")) != Z3_OK) return st;
    if (nmaps > 1) {
        hipLaunchKernelGGL(k_group_values, dim3(grid_for(idx->n)), dim3(256), 0, s, idx->n, nmaps, idx->d_band,
                           idx->d_bands, idx->d_v, idx->d_vgrp);
        const int ldv = batch_ldv(nmaps);
        const int64_t nt = idx->n * ldv;
        const int64_t g = (nt + 255) / 256 < (1 << 20) ? (nt + 255) / 256 : (1 << 20);
        hipLaunchKernelGGL(k_value_matrix, dim3((unsigned)g), dim3(256), 0, s, idx->n, nmaps, ldv, idx->d_band,
                           idx->d_bands, idx->d_v, idx->d_vmat64, idx->d_vmat32);
        if ((st = check_launch("k_group_values/k_value_matrix")) != Z3_OK) return st;
    }
    return Z3_OK;
}

z3_status update_values_impl(z3_index idx, const double *x, hipStream_t s)
{
    return fill_values(idx, idx->nmaps, x, s);
}

z3_status set_values_impl(z3_index idx, int nmaps, const double *x, hipStream_t s)
{
    z3_status st;
    (void)hipStreamSynchronize(s);  // earlier work may still read the old values
    if (idx->d_v) { (void)hipFree(idx->d_v); idx->d_v = nullptr; }
    if (idx->d_rec) { (void)hipFree(idx->d_rec); idx->d_rec = nullptr; }
    if (idx->d_vgrp) { (void)hipFree(idx->d_vgrp); idx->d_vgrp = nullptr; }
    if (idx->d_vmat64) { (void)hipFree(idx->d_vmat64); idx->d_vmat64 = nullptr; }
    if (idx->d_vmat32) { (void)hipFree(idx->d_vmat32); idx->d_vmat32 = nullptr; }
    idx->nmaps = 0;
    idx->ngroups = 0;
    for (auto &row : idx->batch_shape_tuned)
        for (int &t : row) t = 0;
    size_t cnt = (size_t)nmaps * (size_t)idx->n;
    if ((st = dalloc(&idx->d_v, cnt, "alloc values")) != Z3_OK) return st;
    if ((st = dalloc(&idx->d_rec, 2 * cnt, "alloc records")) != Z3_OK) return st;
    if (nmaps > 1) {
        const int ng = (nmaps + kMapGroup - 1) / kMapGroup;
        if ((st = dalloc(&idx->d_vgrp, (size_t)ng * 2 * idx->n * kMapGroup, "alloc grouped values")) != Z3_OK)
            return st;
        idx->ngroups = ng;
        const int ldv = batch_ldv(nmaps);
        if ((st = dalloc(&idx->d_vmat64, (size_t)2 * idx->n * ldv, "alloc value matrix")) != Z3_OK) return st;
        if ((st = dalloc(&idx->d_vmat32, (size_t)2 * idx->n * ldv, "alloc value matrix")) != Z3_OK) return st;
    }
    if ((st = fill_values(idx, nmaps, x, s)) != Z3_OK) return st;
    idx->nmaps = nmaps;
    return Z3_OK;
}

}  // namespace z3
