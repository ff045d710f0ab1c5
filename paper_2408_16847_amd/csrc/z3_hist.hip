// Angular-histogram multipoles: the picture the complexity discussion of the "3PCF binned
// estimator" subsection draws of the method -- histograms around each pivot in radial and
// n_phi angular bins, then a Fourier transform over the angular bins -- as an estimator.
//
// Every pair of radial bin b whose bearing lies in angular bin k = [k dphi, (k+1) dphi)
// (dphi = 2 pi / n_phi, bearings from local north towards east) adds w_j x_j to H_{b,k}; the
// multipoles take each pair at its bin centre:
//     a_{m,b} = sum_k H_{b,k} exp(-i m (k + 1/2) dphi),   m <= m_max < n_phi / 2,
// so the per-pair cost no longer grows with m_max (the direct kernel's does, by 4 FP64
// operations per multipole), and m_max is no longer bounded by the direct kernel's registers.
//
// The angular bin is decided exactly, against the caller's FP64 boundary table
// D_k = (cos k dphi, sin k dphi): bin k iff  c_k u2 - s_k u1 >= 0  and
// c_{k+1} u2 - s_{k+1} u1 < 0, where u1, u2 are the separation's components on the
// unnormalised local north N = (-z x, -z y, 1 - z^2) (x-axis fallback at the poles) and east
// E = N x r_p, each dot product summed as (x + y) + z with every operation rounded on its own
// (this file is compiled with -ffp-contract=off).  An FP32 arctangent, accurate to 2e-5 rad,
// decides every bearing farther than 5e-5 rad from a boundary; the others take the sign
// tests, which confirm the estimate or move it to the neighbouring bin.
//
// Work decomposition: blocks of four waves; LPP lanes per pivot (LPP = 1..16 grows with
// n_phi, so that a wave's histogram stays within 9 KiB of LDS and 4 waves per SIMD fit),
// 64 / LPP consecutive index-order pivots per wave, the same band windows, records and
// one-ahead record requests as k_multipoles.  Lane q of a pivot takes the candidates
// q, q + LPP, ... of each window and sums runs of consecutive pairs in one angular bin in
// registers, adding a run into the pivot's row of the wave's LDS histogram [n_phi][64/LPP+1]
// with an FP64 LDS atomic when the bin changes (the order of the adds is fixed by the
// program and the lane order, so results are reproducible).  After the bin's windows the
// pivot's lanes split its multipoles (m = q, q + LPP, ...) and form each from the pivot's
// row, a_m = e^{-i m dphi/2} sum_k H_k e^{-i m k dphi}, by Clenshaw's recurrence over the
// angular bins (one FMA and one subtraction per bin and multipole; the constants come from
// an LDS table of (cos, sin)(pi j / n_phi)).  Sums stay in FP64 on both precision paths;
// the mixed path stores the multipoles in FP32.
#include "z3_internal.h"
#include "z3_device.h"

namespace z3 {

struct HistArgs {
    const double *px, *py, *pz;   // index-order positions (the pivots)
    const double4 *rec;           // doubled-band records {x, y, z, w x} of the map
    const double *wdbl;           // doubled-band weights, or null when all weights are 1
    const int *cell_start;
    const Band *bands;
    int nbands;
    double inv_h;
    const EdgeTab *edges;
    int nb;
    int64_t p0, p1;
    int n_phi;
    float phi_scale;              // n_phi / (2 pi)
    float phi_guard;              // 5e-5 rad in units of angular bins
    const double2 *bounds;        // [n_phi] boundary directions (cos, sin) of the angular bins
    const double2 *tab;           // [2 n_phi] (cos, sin)(pi j / n_phi)
    int m_max;
    int norm;
    void *A;                      // [m_max+1][2][nb][ldA] FP64 or FP32, or null
    int64_t ldA;
    double *W;
    int64_t *counts;              // [nb][ldA] pairs per (pivot, bin), or null
    int *counts_phi;              // [nb][n_phi][ldA] pairs per (pivot, bin, angular bin), or null
    uint64_t *pair_total;
    int nblocks;
};

// Multipoles per lane and pass of the transform.  The lanes-per-pivot choice below keeps
// n_phi / LPP <= 18, and m_max < n_phi / 2, so each lane's share of the m_max + 1
// multipoles is at most 9: one pass.
constexpr int kHistMC = 9;

__device__ __forceinline__ bool left_of(const double2 *D, int k, double u1, double u2)
{
    const double2 d = D[k];
    const double a = d.x * u2;
    const double b = d.y * u1;
    return a - b >= 0.0;
}

// The angular bin by the exact rule, starting from the estimate k: the signs "left of
// boundary k" form one circular run, so the bin (the run's end) is reached by stepping
// towards it; at most n steps.
__device__ __forceinline__ int exact_angular_bin(const double2 *D, int n, int k, double u1, double u2)
{
    int k1 = k + 1 == n ? 0 : k + 1;
    bool lk = left_of(D, k, u1, u2), lk1 = left_of(D, k1, u1, u2);
    for (int it = 0; it < n && !(lk && !lk1); ++it) {
        if (!lk) {
            k1 = k;
            k = k == 0 ? n - 1 : k - 1;
            lk1 = lk;
            lk = left_of(D, k, u1, u2);
        } else {
            k = k1;
            k1 = k1 + 1 == n ? 0 : k1 + 1;
            lk = lk1;
            lk1 = left_of(D, k1, u1, u2);
        }
    }
    return k;
}

// Estimate of the angular bin from an FP32 arctangent of (v1, v2), the tangent components
// in any FP64 rounding (they differ from the exact rule's by ~1e-16 rad): octant reduction
// and the odd polynomial of Abramowitz & Stegun 4.4.49 on [0, 1] (error <= 1e-5 rad); with
// the FP32 rounding of v1, v2, of the reciprocal and of the octant arithmetic the estimate
// is within 2e-5 rad of the bearing.  Returns the bin, and sets `sure` when the bearing lies
// farther than `guard` (5e-5 rad, in bins) from the nearest boundary, where the exact rule
// gives the same bin.  (v1, v2) = 0 cannot be a pair in range; it would give a NaN estimate,
// which is never sure.
__device__ __forceinline__ int angular_estimate(int n, float scale, float guard, double v1, double v2, bool &sure)
{
    const float f1 = (float)v1, f2 = (float)v2;
    const float ax = fabsf(f1), ay = fabsf(f2);
    const float mn = fminf(ax, ay), mx = fmaxf(ax, ay);
    const float t = mn * __builtin_amdgcn_rcpf(mx);
    const float t2 = t * t;
    const float at = t * fmaf(t2, fmaf(t2, fmaf(t2, fmaf(t2, 0.0208351f, -0.0851330f), 0.1801410f), -0.3302995f),
                              0.9998660f);
    float ph = ay > ax ? 1.57079633f - at : at;
    ph = f1 < 0.0f ? 3.14159265f - ph : ph;
    ph = f2 < 0.0f ? 6.28318531f - ph : ph;
    const float q = ph * scale;  // >= 0
    const int k = min((int)q, n - 1);
    const float fr = q - (float)k;
    sure = fr > guard && fr < 1.0f - guard;
    return k;
}

// LDS layout of a block of kHistWaves waves with LPP lanes per pivot (G = 64 / LPP pivots per
// wave): per wave a histogram H [n_phi][G + 1] FP64 (row stride G + 1, odd, so that lanes of
// one pivot adding into different angular bins mostly hit different banks) and, with
// per-cell counts, C [n_phi][G + 1] int32; per block the boundary table D [n_phi] and the
// phase table T [2 n_phi] (double2).
constexpr int kHistWaves = 4;

__host__ __device__ constexpr int hist_row(int lpp) { return kWave / lpp + 1; }

size_t hist_lds_bytes(int n_phi, bool counts, int lpp)
{
    const size_t row = (size_t)hist_row(lpp) * n_phi;
    return kHistWaves * row * (sizeof(double) + (counts ? sizeof(int) : 0)) + 3 * (size_t)n_phi * sizeof(double2);
}

// Lanes per pivot for n_phi angular bins: the smallest power of two that keeps a wave's
// histogram within Z3_HIST_WAVE_LDS bytes (9 KiB: LDS then admits the 16 waves per CU, 4 per
// SIMD, that the register budget allows).
#ifndef Z3_HIST_WAVE_LDS
#define Z3_HIST_WAVE_LDS 9216
#endif
int hist_lanes_per_pivot(int n_phi)
{
    int lpp = 1;
    while (lpp < 16 && (size_t)n_phi * (kWave / lpp) * sizeof(double) > (size_t)Z3_HIST_WAVE_LDS) lpp *= 2;
    return lpp;
}

template <bool F32OUT, bool CNT, int LPP>
__global__ __launch_bounds__(kHistWaves * kWave) __attribute__((amdgpu_waves_per_eu(4)))
void k_multipoles_hist(HistArgs a)
{
    constexpr int G = kWave / LPP;     // pivots per wave
    constexpr int HS = hist_row(LPP);  // histogram row stride (doubles)
    extern __shared__ double smem[];
    const int n = a.n_phi;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int pl = lane / LPP, q = lane % LPP;  // pivot slot in the wave, lane within the pivot
    double *H = smem + (size_t)wave * n * HS;                                    // [n][HS]
    double2 *D = reinterpret_cast<double2 *>(smem + (size_t)kHistWaves * n * HS);  // [n]
    double2 *T = D + n;                                                          // [2n]
    int *C = reinterpret_cast<int *>(T + 2 * n) + (size_t)wave * n * HS;         // [n][HS] (CNT)
    for (int k = threadIdx.x; k < n; k += kHistWaves * kWave) D[k] = a.bounds[k];
    for (int j = threadIdx.x; j < 2 * n; j += kHistWaves * kWave) T[j] = a.tab[j];
    __syncthreads();

    const int lb = xcd_block(blockIdx.x, a.nblocks);
    const int64_t p = a.p0 + ((int64_t)lb * kHistWaves + wave) * G + pl;
    const bool valid = p < a.p1;
    const int64_t pp = valid ? p : a.p1 - 1;  // idle lanes shadow the last pivot
    const double xp = a.px[pp], yp = a.py[pp], zp = a.pz[pp];
    const double sinth = sqrt(xp * xp + yp * yp);
    const double th = atan2(sinth, zp);
    double ph = atan2(yp, xp);
    if (ph < 0.0) ph += kTwoPi;
    double sh, ch;
    sincos(0.5 * th, &sh, &ch);
    const float inv_sp = sinth > 0.0 ? (float)(1.0 / sinth) : INFINITY;
    const float phf = (float)ph;
    // unnormalised local north and east of the bin decision
    double nx = -zp * xp, ny = -zp * yp, nz = 1.0 - zp * zp;
    const double nn = (nx * nx + ny * ny) + nz * nz;
    if (nn < 1e-24) {
        nx = 1.0 - xp * xp;
        ny = -xp * yp;
        nz = -xp * zp;
    }
    const double ex = ny * zp - nz * yp, ey = nz * xp - nx * zp, ez = nx * yp - ny * xp;

    const int64_t col = p - a.p0;
    const int nb = a.nb;
    const bool unit_w = a.wdbl == nullptr;
    uint64_t my_pairs = 0;

    for (int bin = 0; bin < nb; ++bin) {
        for (int e = lane; e < n * HS; e += kWave) {
            H[e] = 0.0;
            if constexpr (CNT) C[e] = 0;
        }
        // this wave's LDS writes are done before any lane of it adds into the histogram
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        const double elo = a.edges->e[bin], ehi = a.edges->e[bin + 1];
        const double hav_out = a.edges->hav_out[bin + 1], hav_in = a.edges->hav_in[bin];
        int klo, khi;
        band_range(th, a.edges->rad_out[bin + 1], a.inv_h, a.nbands, klo, khi);
        // wpend: the weight of the lane's previous pair, added at its next pair (or after the
        // bin), so that its load overlaps a candidate's work; the additions keep their order
        double Wb = 0.0, wpend = 0.0;
        int cnt = 0;
        // run of consecutive pairs (of this lane) in one angular bin, summed in registers and
        // added to the pivot's histogram row by an LDS atomic when the bin changes
        int krun = 0, crun = 0;
        double vrun = 0.0;
        // the pairs of one band: the pivot's windows (s0, l0) and (s1, l1) of band bd
        auto walk = [&](const Band &bd, int s0, int l0, int s1, int l1) __attribute__((always_inline)) {
            const int base = 2 * bd.pt_start;
            const __amdgpu_buffer_rsrc_t rband = buffer_view(a.rec + base, (uint32_t)bd.npts * 64u);
            // and its doubled weights (8 B per record: byte offset = record offset / 4)
            const __amdgpu_buffer_rsrc_t wband = buffer_view(unit_w ? nullptr : a.wdbl + base,
                                                             unit_w ? 0u : (uint32_t)bd.npts * 16u);
            auto cand = [&](const double4 &r, uint32_t o) __attribute__((always_inline)) {
                const double dx = r.x - xp, dy = r.y - yp, dz = r.z - zp;
                const double d2 = (dx * dx + dy * dy) + dz * dz;
                if (d2 >= elo && d2 < ehi) {
                    cnt += 1;
                    if (!unit_w) {
                        Wb += wpend;
                        wpend = load_f64(wband, o >> 2);
                    }
                    bool sure;
                    int k = angular_estimate(n, a.phi_scale, a.phi_guard, fma(dx, nx, fma(dy, ny, dz * nz)),
                                             fma(dx, ex, fma(dy, ey, dz * ez)), sure);
                    if (!sure) {
                        // the exact rule's tangent components: every product and sum rounded
                        // on its own (this file is compiled with -ffp-contract=off)
                        const double u1 = (dx * nx + dy * ny) + dz * nz;
                        const double u2 = (dx * ex + dy * ey) + dz * ez;
                        k = exact_angular_bin(D, n, k, u1, u2);
                    }
                    if (k != krun) {
                        if (crun) {
                            atomicAdd(&H[krun * HS + pl], vrun);
                            if constexpr (CNT) atomicAdd(&C[krun * HS + pl], crun);
                        }
                        krun = k;
                        vrun = 0.0;
                        crun = 0;
                    }
                    vrun += r.w;
                    crun += 1;
                }
            };
            // lane q of a pivot takes the candidates q, q + LPP, q + 2 LPP, ... of each window
            constexpr uint32_t step = 32u * LPP;
#pragma unroll
            for (int seg = 0; seg < 2; ++seg) {
                uint32_t off = (uint32_t)((seg == 0 ? s0 : s1) + q) * 32u;
                const uint32_t oend = (uint32_t)((seg == 0 ? s0 + l0 : s1 + l1)) * 32u;
                // record requested one candidate ahead, two record registers in turn; past
                // the window a request reads an unused record of the band (or zeros past it)
                double4 ra = load_record(rband, off < oend ? off : 0u);
                for (; off < oend; off += 2u * step) {
                    const double4 rb = load_record(rband, off + step);
                    cand(ra, off);
                    if (off + step >= oend) break;
                    ra = load_record(rband, off + 2u * step);
                    cand(rb, off + step);
                }
            }
        };
        if constexpr (LPP < 4) {
            // every lane computes its pivot's windows one band at a time from the band's
            // wave-uniform record
            for (int kb = klo; kb <= khi; ++kb) {
                const Band bd = a.bands[kb];
                if (bd.npts == 0) continue;
                int s0, l0, s1, l1;
                band_window(bd, a.cell_start, th, sh, ch, inv_sp, phf, hav_out, hav_in, s0, l0, s1, l1);
                walk(bd, s0, l0, s1, l1);
            }
        } else {
            // lane q of each pivot computes the pivot's windows in band kb0 + q; the pivot's
            // lanes then walk these LPP bands in turn, each band's windows taken from the lane
            // that computed them (the window arithmetic once per pivot and band, where one band
            // at a time would repeat it on every lane of the pivot)
            for (int kb0 = klo; kb0 <= khi; kb0 += LPP) {
                int w0 = 0, wl0 = 0, w1 = 0, wl1 = 0;
                if (kb0 + q <= khi) {
                    const Band bq = a.bands[kb0 + q];
                    if (bq.npts > 0)
                        band_window(bq, a.cell_start, th, sh, ch, inv_sp, phf, hav_out, hav_in, w0, wl0, w1, wl1);
                }
                const int nband = min(LPP, khi - kb0 + 1);
                for (int b = 0; b < nband; ++b) {
                    const Band bd = a.bands[kb0 + b];
                    if (bd.npts == 0) continue;
                    const int src = (lane & ~(LPP - 1)) + b;
                    walk(bd, __shfl(w0, src, kWave), __shfl(wl0, src, kWave), __shfl(w1, src, kWave),
                         __shfl(wl1, src, kWave));
                }
            }
        }
        if (crun) {
            atomicAdd(&H[krun * HS + pl], vrun);
            if constexpr (CNT) atomicAdd(&C[krun * HS + pl], crun);
        }
        if (valid) my_pairs += (uint64_t)cnt;
        Wb += wpend;
        // the pivot's pair count and weight sum over its LPP lanes (a butterfly: every lane of
        // the pivot ends with the same, fixed-order sum)
#pragma unroll
        for (int o = 1; o < LPP; o <<= 1) {
            cnt += __shfl_xor(cnt, o, kWave);
            if (!unit_w) Wb += __shfl_xor(Wb, o, kWave);
        }
        if (unit_w) Wb = (double)cnt;
        double inv = 1.0;
        if (a.norm == Z3_NORM_BIN) inv = Wb > 0.0 ? 1.0 / Wb : 0.0;
        // every lane's atomics into the wave's histogram are done before it is read
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        // Fourier sum over the angular bins at their centres,
        //   a_m = e^{-i m dphi/2} sum_k H_k z^k,  z = e^{-i w}, w = m dphi,
        // by Clenshaw's recurrence over k (backwards): b_k = H_k + 2 cos(w) b_{k+1} - b_{k+2},
        // then sum_k H_k cos(k w) = b_0 - cos(w) b_1 and sum_k H_k sin(k w) = sin(w) b_1: one FMA
        // and one subtraction per (k, m); lane q of a pivot takes m = q, q + LPP, ..., kHistMC
        // of them per pass over the pivot's row
        if (a.A) {
            for (int m0 = q; m0 <= a.m_max; m0 += kHistMC * LPP) {
                double tc[kHistMC], b1[kHistMC], b2[kHistMC];
#pragma unroll
                for (int i = 0; i < kHistMC; ++i) {
                    const int m = m0 + i * LPP <= a.m_max ? m0 + i * LPP : 0;
                    tc[i] = 2.0 * T[2 * m].x;  // 2 cos(m dphi) = 2 cos(pi 2m / n_phi)
                    b1[i] = 0.0;
                    b2[i] = 0.0;
                }
                for (int k = n - 1; k >= 0; --k) {
                    const double h = H[k * HS + pl];
#pragma unroll
                    for (int i = 0; i < kHistMC; ++i) {
                        const double b0 = fma(tc[i], b1[i], h) - b2[i];
                        b2[i] = b1[i];
                        b1[i] = b0;
                    }
                }
                if (valid) {
#pragma unroll
                    for (int i = 0; i < kHistMC; ++i) {
                        const int m = m0 + i * LPP;
                        if (m > a.m_max) break;
                        const double2 cw = T[2 * m], hw = T[m];  // (cos, sin)(m dphi), (cos, sin)(m dphi / 2)
                        const double pr = b1[i] - cw.x * b2[i], pi = -cw.y * b2[i];  // sum_k H_k z^k
                        // a_m = e^{-i m dphi / 2} (pr + i pi) = Y - i Z
                        const double Y = hw.x * pr + hw.y * pi;
                        const double Z = hw.y * pr - hw.x * pi;
                        const double re = Y * inv;
                        const double im = m == 0 ? 0.0 : -Z * inv;
                        const size_t ore = ((size_t)(2 * m) * nb + bin) * (size_t)a.ldA + col;
                        const size_t oim = ((size_t)(2 * m + 1) * nb + bin) * (size_t)a.ldA + col;
                        if constexpr (F32OUT) {
                            static_cast<float *>(a.A)[ore] = (float)re;
                            static_cast<float *>(a.A)[oim] = (float)im;
                        } else {
                            static_cast<double *>(a.A)[ore] = re;
                            static_cast<double *>(a.A)[oim] = im;
                        }
                    }
                }
            }
        }
        if (valid) {
            const size_t ob = (size_t)bin * (size_t)a.ldA + col;
            if (q == 0) {
                if (a.W) a.W[ob] = Wb;
                if (a.counts) a.counts[ob] = cnt;
            }
            if constexpr (CNT) {
                for (int k = q; k < n; k += LPP)
                    a.counts_phi[((size_t)bin * n + k) * (size_t)a.ldA + col] = C[k * HS + pl];
            }
        }
        // the histogram is read by every lane of the wave before the next bin clears it
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
    }

    if (a.pair_total) {
        const uint64_t tot = wave_sum_u64(my_pairs);
        if (lane == 0 && tot) atomicAdd((unsigned long long *)a.pair_total, (unsigned long long)tot);
    }
}

template <bool F32OUT, bool CNT>
static void launch_hist_lpp(int lpp, dim3 grid, size_t lds, hipStream_t s, const HistArgs &a)
{
    const dim3 block(kHistWaves * kWave);
    switch (lpp) {
    case 1: hipLaunchKernelGGL((k_multipoles_hist<F32OUT, CNT, 1>), grid, block, lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_multipoles_hist<F32OUT, CNT, 2>), grid, block, lds, s, a); break;
    case 4: hipLaunchKernelGGL((k_multipoles_hist<F32OUT, CNT, 4>), grid, block, lds, s, a); break;
    case 8: hipLaunchKernelGGL((k_multipoles_hist<F32OUT, CNT, 8>), grid, block, lds, s, a); break;
    default: hipLaunchKernelGGL((k_multipoles_hist<F32OUT, CNT, 16>), grid, block, lds, s, a); break;
    }
}

z3_status launch_multipoles_hist(const z3_index_s *idx, int map, int m_max, int prec, int norm, int64_t p0,
                                 int64_t p1, void *A, int64_t ldA, double *W, int64_t *counts, int *counts_phi,
                                 uint64_t *pair_total, hipStream_t s)
{
    if (idx->n_phi < 4 || !idx->d_phi_bounds || !idx->d_phi_tab)
        return fail(Z3_ERR_INVALID_ARG, "angular bins not set on this index (z3_index_set_phi_bins)");
    if (m_max < 0 || 2 * m_max >= idx->n_phi)
        return fail(Z3_ERR_INVALID_ARG, "m_max=%d needs m_max < n_phi / 2 = %d / 2", m_max, idx->n_phi);
    const int lpp = hist_lanes_per_pivot(idx->n_phi);
    const int64_t per_block = (int64_t)kHistWaves * (kWave / lpp);
    const int64_t nblk = (p1 - p0 + per_block - 1) / per_block;
    if (nblk > 0x7fffffff) return fail(Z3_ERR_OVERFLOW, "too many pivot blocks");
    if (nblk == 0) return Z3_OK;
    const bool cnt = counts_phi != nullptr;
    const size_t lds = hist_lds_bytes(idx->n_phi, cnt, lpp);
    int dev = 0, lds_max = 0;
    z3_status st = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st == Z3_OK)
        st = check_hip(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
                       "hipDeviceGetAttribute");
    if (st != Z3_OK) return st;
    if (lds > (size_t)lds_max)
        return fail(Z3_ERR_UNSUPPORTED, "n_phi=%d needs %zu bytes of LDS per block%s, the device offers %d",
                    idx->n_phi, lds, cnt ? " with per-cell counts" : "", lds_max);
    HistArgs a;
    a.px = idx->d_x; a.py = idx->d_y; a.pz = idx->d_z;
    a.rec = idx->d_rec + (size_t)map * 2 * idx->n;
    a.wdbl = idx->unit_w ? nullptr : idx->d_wdbl;
    a.cell_start = idx->d_cell_start;
    a.bands = idx->d_bands;
    a.nbands = idx->nbands;
    a.inv_h = 1.0 / idx->band_h;
    a.edges = idx->d_edges;
    a.nb = idx->nbins;
    a.p0 = p0; a.p1 = p1;
    a.n_phi = idx->n_phi;
    a.phi_scale = (float)((double)idx->n_phi / kTwoPi);
    a.phi_guard = (float)(5e-5 * (double)idx->n_phi / kTwoPi);
    a.bounds = idx->d_phi_bounds;
    a.tab = idx->d_phi_tab;
    a.m_max = m_max;
    a.norm = norm;
    a.A = A; a.ldA = ldA;
    a.W = W; a.counts = counts; a.counts_phi = counts_phi; a.pair_total = pair_total;
    a.nblocks = (int)nblk;
    const bool f32 = prec == Z3_PREC_MIXED;
    hipEvent_t ev0;
    profile_begin(s, &ev0);
    const dim3 grid((unsigned)nblk);
    if (f32) {
        if (cnt) launch_hist_lpp<true, true>(lpp, grid, lds, s, a);
        else launch_hist_lpp<true, false>(lpp, grid, lds, s, a);
    } else {
        if (cnt) launch_hist_lpp<false, true>(lpp, grid, lds, s, a);
        else launch_hist_lpp<false, false>(lpp, grid, lds, s, a);
    }
    st = check_launch("k_multipoles_hist");
    profile_end(s, ev0);
    return st;
}

}  // namespace z3
