// External pivots in the index's band order.
//
// The multipole kernel gives each wave 64 consecutive pivots and walks, for every bin, the
// union of their band ranges; its lanes read neighbouring records when their pivots are
// neighbours.  A caller's catalogue in no spatial order (a galaxy survey in the order of its
// target list, say) puts far-apart pivots in one wave: the band union then covers most of
// the sky and every lane reads its own cache lines, about 24 times the time of the same
// pivots in HEALPix RING order on the Nside 512 map.  The call's pivots are therefore sorted
// once by a key of the index's grid -- band (colatitude, or y on a plane), then one of 256
// cells along the band -- with a stable radix sort, which keeps the caller's order inside a
// cell; each pivot chunk then gathers its positions and values in that order before the
// multipole and contraction launches (a chunk is a contiguous run of the sorted pivots, so it
// is as dense on the sky as the catalogue).  zeta is a sum over the pivots, so
// only the order of its FP64 additions changes; the sort is stable, so repeated calls give
// identical results.
#include "z3_internal.h"

#include <rocprim/device/device_radix_sort.hpp>

namespace z3 {

// Sort key: band index in the high bits, position along the band in [0, 1) quantised to the
// `fb` low bits (at most 256 cells per band).  Non-finite pivots get band 0, position 0 (their pairs are still counted by
// the kernel's own tests).
__global__ void k_pivot_keys(Pivots piv, int64_t c0, int64_t len, int planar, double inv_h, double x0, double y0,
                             double sx, int nbands, int fb, uint32_t *key, int *val)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    const double x = piv.x[c0 + i], y = piv.y[c0 + i];
    double band, t;
    if (planar) {
        band = (y - y0) * inv_h;
        t = (x - x0) * sx;  // the strips' cell coordinate, in [0, 2 pi)
    } else {
        const double z = piv.z[c0 + i];
        band = atan2(sqrt(x * x + y * y), z) * inv_h;
        t = atan2(y, x);
        if (t < 0.0) t += kTwoPi;
    }
    t *= 1.0 / kTwoPi;
    const double bmax = (double)(nbands - 1);
    const int k = band >= 0.0 ? (int)fmin(floor(band), bmax) : 0;  // NaN: 0
    const double scale = (double)(1u << fb);
    const uint32_t q = t >= 0.0 ? (uint32_t)fmin(floor(t * scale), scale - 1.0) : 0u;
    key[i] = ((uint32_t)k << fb) | q;
    val[i] = (int)i;
}

__global__ void k_gather_pivots(const int *perm, int64_t len, Pivots piv, int64_t p0, const double *w,
                                const double *x, double *gx, double *gy, double *gz, double *gv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    const int64_t j = p0 + perm[i];
    gx[i] = piv.x[j];
    gy[i] = piv.y[j];
    gz[i] = piv.z[j];
    gv[i] = w ? w[j] * x[j] : x[j];  // v = w x, as for the index's own pivots
}

z3_status sort_pivots(const z3_index_s *idx, Pivots piv, int64_t p0, int64_t len, int *perm, hipStream_t s)
{
    if (len <= 0) return Z3_OK;
    int bits = 1;
    while (bits < 26 && (1 << bits) < idx->nbands) ++bits;
    // 256 cells along each band: a caller's coherent order (HEALPix RING: one ring after the
    // other) survives inside a cell, where the stable sort keeps it, and an incoherent one is
    // cut into compact patches
    const int fb = 32 - bits < 8 ? 32 - bits : 8;
    void *wk = nullptr, *wt = nullptr;
    const size_t n = (size_t)len;
    z3_status st = scratch_alloc(&wk, n * 3 * sizeof(uint32_t), s);
    if (st != Z3_OK) return st;
    uint32_t *k_in = static_cast<uint32_t *>(wk), *k_out = k_in + n;
    int *v_in = reinterpret_cast<int *>(k_out + n);
    size_t tbytes = 0;
    st = check_hip(rocprim::radix_sort_pairs(nullptr, tbytes, k_in, k_out, v_in, perm, n, 0, 32, s),
                   "pivot sort size");
    // a non-null temporary buffer: a null one only asks for its size
    if (st == Z3_OK) st = scratch_alloc(&wt, tbytes > 256 ? tbytes : 256, s);
    if (st == Z3_OK) {
        hipLaunchKernelGGL(k_pivot_keys, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, piv, p0, len,
                           idx->planar ? 1 : 0, 1.0 / idx->band_h, idx->plane_x0, idx->plane_y0, idx->plane_sx,
                           idx->nbands, fb, k_in, v_in);
        st = check_launch("k_pivot_keys");
    }
    if (st == Z3_OK)
        st = check_hip(rocprim::radix_sort_pairs(wt, tbytes, k_in, k_out, v_in, perm, n, 0, 32, s), "pivot sort");
    scratch_free(wt, s);
    scratch_free(wk, s);
    return st;
}

z3_status gather_pivots(const int *perm, int64_t len, Pivots piv, int64_t p0, const double *w, const double *x,
                        double *gx, double *gy, double *gz, double *gv, hipStream_t s)
{
    if (len <= 0) return Z3_OK;
    hipLaunchKernelGGL(k_gather_pivots, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, perm, len, piv, p0, w,
                       x, gx, gy, gz, gv);
    return check_launch("k_gather_pivots");
}

}  // namespace z3
