// Internal declarations of libzeta3 (not part of the ABI).
#pragma once

#include <vector>

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "zeta3.h"

#define Z3_API extern "C" __attribute__((visibility("default")))

namespace z3 {

constexpr int kBlock = 256;      // threads per block of the multipole kernel (4 wave64s)
#ifndef Z3_CELLS_PER_POINT
#define Z3_CELLS_PER_POINT 4
#endif
constexpr int kCellsPerPoint = Z3_CELLS_PER_POINT;  // longitude cells per point of a band (tuning)
constexpr int kMapGroup = 4;       // maps carried per lane by the many-map kernel
constexpr int kWave = 64;
// Largest | |r|^2 - 1 | accepted for catalogue positions on the sphere (z3_build_index)
constexpr double kMaxNormDev = 1e-10;
// Pivots whose length differs from 1 by more than this get windows rescaled to their length
constexpr double kPivotNormTol = 4e-11;
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;

// One latitude band of the sky-cell grid.  A band holds the points whose colatitude
// lies in [k H, (k+1) H); inside the band the points are bucketed into `ncell` equal
// longitude cells and sorted by cell.  th_lo/th_hi are the smallest and largest
// colatitude actually present, and the window computation uses their half-angle
// sines and cosines.
struct Band {
    double sh_lo, ch_lo, sh_hi, ch_hi;  // sin, cos of th_lo/2 and th_hi/2
    double th_lo, th_hi;                // colatitude range of the band's points
    float inv_smin, inv_smax;           // 1 / min and 1 / max of sin(theta) over [th_lo, th_hi]
    float cells_per_rad;                // ncell / (2 pi)
    int pt_start, npts;                 // first index-order point and count
    int cell_off, ncell;                // first global cell id and count
    int pad_;
};

// Edge tables derived from the caller's chord-squared edges.  hav = E/4 = sin^2(theta/2).
struct EdgeTab {
    double e[Z3_MAX_NBINS + 1];        // chord-squared edges (exact copy)
    double hav_out[Z3_MAX_NBINS + 1];  // E/4 enlarged by a rounding guard (outer windows)
    double hav_in[Z3_MAX_NBINS + 1];   // E/4 reduced by a rounding guard (inner exclusion)
    double rad_out[Z3_MAX_NBINS + 1];  // angular radius 2 asin(sqrt(E)/2), enlarged
};

}  // namespace z3

struct z3_index_s {
    int device = 0;
    int64_t n = 0;
    int nbins = 0;
    double band_h = 0.0;
    int nbands = 0;
    int64_t ncells = 0;
    z3::EdgeTab edges{};
    z3::EdgeTab *d_edges = nullptr;   // device copy
    z3::Band *d_bands = nullptr;      // [nbands]
    int *d_cell_start = nullptr;      // [ncells + 1], index-order point positions
    double *d_x = nullptr, *d_y = nullptr, *d_z = nullptr, *d_w = nullptr;  // [n], index order
    int *d_perm = nullptr;            // [n] original catalogue index
    int *d_band = nullptr;            // [n] band of each index-order point
    bool unit_w = true;               // all weights are 1 (W_{p,b} = N_{p,b})
    // pivots on a plane: points (x, y, 0); bands are strips of y - plane_y0, and the
    // longitude coordinate of the cells is (x - plane_x0) * plane_sx in [0, 2 pi)
    bool planar = false;
    double plane_x0 = 0.0, plane_y0 = 0.0, plane_sx = 0.0;
    // neighbour records in "doubled band" order: band k occupies [2 s_k, 2 s_k + 2 n_k)
    // and holds its n_k points twice, so every longitude window, wrapped or not, is one
    // contiguous range
    double *d_wdbl = nullptr;         // [2n] weights (only when !unit_w)
    int *d_permdbl = nullptr;         // [2n] original catalogue index
    int nmaps = 0;
    double *d_v = nullptr;            // [nmaps][n] w * x in index order
    double4 *d_rec = nullptr;         // [nmaps][2n] {x, y, z, w * x}
    int ngroups = 0;                  // map groups of kMapGroup for the many-map kernel
    double *d_vgrp = nullptr;         // [ngroups][2n][kMapGroup] w * x, doubled bands
    // per-record value matrices of the MFMA many-map kernel: [2n][ldv] w * x, doubled
    // bands, maps padded with zeros to ldv = a multiple of 32
    double *d_vmat64 = nullptr;
    float *d_vmat32 = nullptr;
    int batch_shape_forced = -1;      // -1: autotune; else a block shape id
    int batch_shape_tuned[2][Z3_MAX_MMAX + 1] = {};  // [prec][m_max] -> shape id + 1 (0 = not yet)
    // workspace of calls captured into a HIP graph (z3_index_prepare_capture): captured calls
    // take their chunk buffers from here instead of allocating
    void *cap_ws = nullptr;
    size_t cap_bytes = 0;
    // earlier, smaller capture workspaces: graphs captured before a reservation grew still
    // point at them, so they are kept (not freed) until z3_index_free
    std::vector<void *> cap_retired;
    // angular bins of the histogram estimator (z3_index_set_phi_bins)
    int n_phi = 0;
    double2 *d_phi_bounds = nullptr;  // [n_phi] boundary directions (cos, sin) of the bins
    double2 *d_phi_tab = nullptr;     // [2 n_phi] (cos, sin)(pi j / n_phi): bin-centre phases
    size_t ws_peak = 0;               // largest scratch total of one eager call on this index
};

namespace z3 {

// Scratch accounting of one API call on an index (z3_api.hip).  While it is alive,
// scratch_alloc either allocates from the library's stream-ordered pool (eager calls; the
// total is recorded in idx->ws_peak) or, when the stream is being captured into a graph,
// hands out consecutive slices of idx->cap_ws (nothing is allocated, scratch_free is a
// no-op), so that the captured kernels point at memory that stays valid for every replay.
struct CallScope {
    CallScope(z3_index idx, hipStream_t s);
    ~CallScope();
    CallScope(const CallScope &) = delete;
    CallScope &operator=(const CallScope &) = delete;
    z3_index idx;
    bool capturing = false;
    size_t used = 0;
    CallScope *prev = nullptr;
};

// While alive on a thread, kernel timing (z3_profile_enable) skips that thread's launches.
struct ProfileMute {
    ProfileMute();
    ~ProfileMute();
};

// error reporting (z3_api.hip)
z3_status fail(z3_status s, const char *fmt, ...);
z3_status check_hip(hipError_t e, const char *what);
z3_status check_launch(const char *what);
// Z3_ERR_OUT_OF_MEMORY if `bytes` exceed the device allocation limit (z3_set_device_alloc_limit)
z3_status alloc_allowed(size_t bytes, const char *what);

// index kernels (z3_index.hip)
z3_status build_index_impl(int64_t n, const double *xyz, const double *w, int nbins,
                           const double *edges, double cell_size, hipStream_t s, z3_index *out,
                           bool planar = false);
z3_status update_values_impl(z3_index idx, const double *x, hipStream_t s);
z3_status set_values_impl(z3_index idx, int nmaps, const double *x, hipStream_t s);
void free_index(z3_index idx);

// multipole kernels (z3_multipoles.hip)
// Pivot positions: either the index's own points (index order) or an external catalogue.
struct Pivots {
    const double *x, *y, *z;
};
z3_status launch_multipoles(const z3_index_s *idx, Pivots piv, int map, int m_max, int prec,
                            int norm, int64_t p0, int64_t p1, void *A, int64_t ldA, double *W,
                            int64_t *counts, uint64_t *idhash, uint64_t *pair_total,
                            hipStream_t s, const double *self_pv = nullptr,
                            double *self_part = nullptr);

// angular-histogram multipoles (z3_hist.hip); counts_phi [nb][n_phi][ldA] or null
z3_status launch_multipoles_hist(const z3_index_s *idx, int map, int m_max, int prec, int norm, int64_t p0,
                                 int64_t p1, void *A, int64_t ldA, double *W, int64_t *counts, int *counts_phi,
                                 uint64_t *pair_total, hipStream_t s);
size_t hist_lds_bytes(int n_phi, bool counts, int lanes_per_pivot);
int hist_lanes_per_pivot(int n_phi);

int batch_ldv(int nmaps);
int batch_num_shapes();
void batch_shape_dims(int shape, int *waves, int *tiles_per_wave);
z3_status batch_shape(z3_index idx, int m_max, int prec, int64_t p0, int64_t p1, hipStream_t s, int *shape);
// stage: [P][nb][nmaps][2 (m+1)] pivot-major buffer the kernel writes (required); A (or
// null): transposed into [map][2 (m+1)][nb][ldA], maps map_stride elements apart
z3_status launch_multipoles_batch(const z3_index_s *idx, int m_max, int prec, int shape, int64_t p0, int64_t p1,
                                  void *stage, void *A, int64_t ldA, size_t map_stride, double *W,
                                  uint64_t *pair_total, hipStream_t s);
// External pivots in the index's band order (z3_pivsort.hip): sort_pivots writes perm [len],
// the stable order of pivots [p0, p0 + len) by band and 256 cells per band; gather_pivots
// copies pivots p0 + perm[i] (i < len) and their values w x (w null: x) into gx, gy, gz, gv.
z3_status sort_pivots(const z3_index_s *idx, Pivots piv, int64_t p0, int64_t len, int *perm, hipStream_t s);
z3_status gather_pivots(const int *perm, int64_t len, Pivots piv, int64_t p0, const double *w, const double *x,
                        double *gx, double *gy, double *gz, double *gv, hipStream_t s);

// Many maps over one set of positions: the MFMA kernel (one block per pivot, every map at
// once) or passes of the register-tiled kernel over the groups of kMapGroup maps.  Measured on
// the Nside 512 map at m_max = 10 (estimator step, multipoles and contraction): a group pass
// costs ~0.148 s (FP64) / ~0.14 s (mixed), so n maps take ~37 / ~35 ms per map; the MFMA
// kernel takes 1.05-1.10 / 0.69-0.72 s for 5 to 16 maps, 1.39 / 0.89 s for 32, 2.06 / 1.33 s
// for 48 and 2.15 / 1.37 s for 64.  The groups are therefore faster up to ~56 maps on the
// FP64 path and ~24 on the mixed one.  A block shape fixed by the caller
// (z3_index_set_batch_shape) selects the MFMA kernel for more than kMapGroup maps.
inline bool many_maps_on_mfma(const z3_index_s *idx, int prec)
{
    if (idx->nmaps <= kMapGroup) return false;
    if (idx->batch_shape_forced >= 0) return true;
    return idx->nmaps > (prec == Z3_PREC_FP64 ? 56 : 24);
}

// Multipoles of the maps of attached group `group` (kMapGroup maps, map_stride elements apart
// in A); only the first `nslots` (1..kMapGroup) are guaranteed written.
z3_status launch_multipoles_maps(const z3_index_s *idx, int group, int nslots, int m_max, int prec, int64_t p0,
                                 int64_t p1, void *A, int64_t ldA, size_t map_stride, double *W,
                                 uint64_t *pair_total, hipStream_t s);

// contraction and small kernels (z3_contract.hip)
z3_status launch_contract(int64_t npiv, int m_max, int nbins, int prec, const void *A,
                          int64_t ldA, const double *piv_v, double *zeta, void *partials,
                          size_t partial_bytes, hipStream_t s);
// nmaps contractions in one launch: map k reads A + k a_stride, piv_v + k v_stride and adds
// into zeta + k z_stride; partials hold nmaps x contract_partial_bytes
z3_status launch_contract_maps(int64_t npiv, int m_max, int nbins, int prec, int nmaps, const void *A, int64_t ldA,
                               size_t a_stride, const double *piv_v, size_t v_stride, double *zeta, size_t z_stride,
                               void *partials, size_t partial_bytes, hipStream_t s);
// the same contraction reading the many-map kernel's pivot-major staging
// [P][nb][nmaps][2 (m+1)]; needs gram_lds_fits
z3_status launch_contract_staged(int64_t npiv, int m_max, int nbins, int prec, int nmaps, const void *stage,
                                 const double *piv_v, size_t v_stride, double *zeta, size_t z_stride, void *partials,
                                 size_t partial_bytes, hipStream_t s);
bool gram_lds_fits(int m_max, int nbins, int prec);
// multi-field contraction: zeta[m][b1][b2] += sum_p v_p X1_m(b1; p) conj(X2_m(b2; p)),
// X1 and X2 in the pivot-minor layout [m+1][2][nbins][ldA]
z3_status launch_contract_cross(int64_t npiv, int m_max, int nbins, int prec, const void *A1, const void *A2,
                                int64_t ldA, const double *piv_v, double *zeta, void *partials,
                                size_t partial_bytes, hipStream_t s);
size_t cross_partial_bytes(int64_t npiv, int m_max, int nbins);
size_t contract_partial_bytes(int64_t npiv, int m_max, int nbins);
z3_status launch_weight_sum(const double *w, int64_t n, double *out, hipStream_t s);
z3_status launch_pivot_values(const double *w, const double *x, int64_t n, double *v, hipStream_t s);
z3_status launch_add_scalar(double *out, double value, hipStream_t s);
z3_status launch_fill(double *p, int64_t n, double value, hipStream_t s);
// zeta[m][b][b] re -= sum over the nw rows of part [nw][nbins] (column b), for m <= m_max
// FFTLog line-of-sight integrals (z3_fftlog.hip): workspace bytes for `chunk` models per
// pass, and the evaluation itself (nu [4] host; every array a device pointer)
size_t fftlog_workspace_bytes(int N, int nchi, int T, int chunk);
z3_status fftlog_impl(int N, const double *Pk, double k_min, double k_max, const double *nu, int nchi, double chi_min,
                      double chi_max, int nmodels, const double *F, int T, const double *theta, double *out,
                      void *ws, int chunk, hipStream_t s);
z3_status launch_self_subtract(const double *part, int64_t nw, int m_max, int nbins, double *zeta,
                               hipStream_t s);

// adjoint (z3_adjoint.hip)
z3_status adjoint_impl(z3_index idx, int map, int m_max, int64_t p0, int64_t p1, const double *G,
                       double scale, double *grad_x, hipStream_t s, int64_t chunk);
z3_status adjoint_maps_impl(z3_index idx, int m_max, int64_t p0, int64_t p1, const double *G,
                            double scale, double *grad_x, hipStream_t s, int64_t chunk);
z3_status launch_finalize(int nmaps, int m_max, int nbins, double *zeta, const double *sum_w,
                          hipStream_t s);
z3_status launch_resum(int m_max, int nbins, const double *zeta, int nphi, const double *phi,
                       double *out, hipStream_t s);

// kernel timing (z3_api.hip)
bool profiling();
void profile_begin(hipStream_t s, hipEvent_t *ev0);
void profile_end(hipStream_t s, hipEvent_t ev0);

// stream-ordered scratch allocations from a library-private pool (memory stays cached)
z3_status scratch_alloc(void **p, size_t bytes, hipStream_t s);
void scratch_free(void *p, hipStream_t s);

}  // namespace z3
