// Ball search + binning + multipole accumulation (eqs. Xm.binned and Ym/Zm.binned).
//
// Work decomposition: one lane per pivot, 64 consecutive index-order pivots per wave
// (neighbouring points of one latitude band, so their neighbour windows overlap and the
// lanes' loads of neighbour points fall on the same cache lines).  Each lane walks the
// radial bins in order; for bin b it visits, band by band, only the longitude window
// that can hold neighbours at chord-squared distance in [E_b, E_{b+1}), and keeps the
// bin's sums in registers:
//
//   Y_m = sum w_j x_j cos(m phi),  Z_m = sum w_j x_j sin(m phi),  W = sum w_j,  N = #pairs
//
// so a_{m,b} = Y_m - i Z_m.  There are no atomics and no cross-lane reductions, and the
// summation order of every (pivot, bin) is fixed, so results are bit-reproducible.
//
// Exactness of the pair decision: d2 = (dx*dx + dy*dy) + dz*dz in FP64 with every
// operation rounded separately (this file is compiled with -ffp-contract=off), compared
// with the caller's FP64 edges.  The longitude windows are conservative (rounding
// guards), so they never drop a pair that the d2 test accepts.
//
// Harmonics: the paper's remark after the binned estimator builds cos(m phi) and
// sin(m phi) from Chebyshev polynomials of cos(phi), so that no trigonometric function is
// evaluated per pair.  Here one second-kind chain per pair, u_k = v U_k(c) with
// U_k = 2 c U_{k-1} - U_{k-2} (c = cos phi, v = w_j x_j), feeds two sums per bin:
//   SU_k = sum u_k  and  SV_k = sum 2 sin(phi) u_k,
// and the bin's epilogue forms Y_m = (SU_m - SU_{m-2}) / 2 (T_m = (U_m - U_{m-2}) / 2,
// U_{-1} = 0) and Z_m = SV_{m-1} / 2 (sin(m phi) = sin(phi) U_{m-1}(c)).  Per pair and m:
// one FMA of the chain, one add and one FMA into the sums, against two FMAs and two adds
// for separate first- and second-kind chains.  Near phi = 0 or pi, U_m ~ m + 1 and the
// difference gives up ~log2(m) bits: ~1e-14 of sum |v| at m = 10 in FP64.
//
// Pivots on a plane (PLANAR): the same loop over a strip x cell grid of (x, y, 0) records;
// the frame is fixed (angles from +y towards +x) and the windows are planar_window's.
//
// Optionally (SELF) the kernel also removes the k = j terms of the contraction's diagonal
// (the overcount the paper points out in the kappa^3 multipole-signal subsection): per
// (pivot, bin) it sums Q = sum_j (w_j x_j)^2 in FP64, forms v_p Q / W^2 (v_p Q for raw
// sums), adds that over the wave in a fixed order and writes one value per (wave, bin).
//
// Precision: both paths form the separation, the exact squared chord, the bearing (an
// FP32-seeded reciprocal square root refined by one FP64 Newton step) and the harmonics in
// FP64 and add them into FP64 bin sums; the mixed path stores the normalised multipoles in
// FP32 for its split-FP32 MFMA contraction.  An FP32 bearing or FP32 recurrences would carry
// an angle error of ~1e-7 per pair, which the m-th harmonic multiplies by m: ~1e-6 at
// m = 10 on fields whose 3PCF is a sum of terms of random sign.  On this hardware the FP32
// vector instructions (packed forms excluded) issue at the FP64 rate, so the FP64 harmonics
// cost the same instructions and are exact to ~1e-15.
#include "z3_internal.h"
#include "z3_device.h"

namespace z3 {

struct MultArgs {
    const double *px, *py, *pz;   // index-order positions (the pivots)
    const double4 *rec;           // doubled-band records {x, y, z, w x} of the map
    const double *wdbl;           // doubled-band weights, or null when all weights are 1
    const int *permdbl;           // doubled-band original indices (neighbour fingerprints)
    const int *cell_start;
    const Band *bands;
    int nbands;
    double inv_h;
    const EdgeTab *edges;
    int nb;
    int64_t p0, p1;
    int norm;
    void *A;
    int64_t ldA;
    double *W;
    int64_t *counts;
    uint64_t *idhash;
    uint64_t *pair_total;
    const double *pv;             // SELF: index-order pivot products w_p x_p
    double *self_part;            // SELF: [waves of the launch][nb] sums of v_p Q / W^2
    double px0, py0, psx;         // PLANAR: plane origin and cell-coordinate scale
    double tiny;                  // kBearingTiny, passed so that it sits in scalar registers
    int nblocks;
};

// Occupancy target of the multipole kernel (waves per SIMD that the register allocation
// aims for).  Measured on MI355X at m_max = 10: 4 waves beat 3 by ~15% despite a couple
// of spilled registers; larger m_max needs more accumulators, so the target drops.
#ifndef Z3_MULT_WAVES_PER_EU
#define Z3_MULT_WAVES_PER_EU 4
#endif
template <int M>
constexpr int mult_waves_per_eu()
{
    return M <= 10 ? Z3_MULT_WAVES_PER_EU : (M <= 13 ? 3 : 2);
}

template <int M, bool F32OUT, bool IDS, bool SELF, bool PLANAR>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(mult_waves_per_eu<M>())))
void k_multipoles(MultArgs a)
{
    // XCD-aware order: hardware hands consecutive block ids to the 8 XCDs in turn;
    // give each XCD a contiguous run of pivot tiles so neighbour data stays in its L2.
    const int nblk = a.nblocks;
    const int bid = blockIdx.x;
    const int per = nblk / 8, rem = nblk % 8;
    const int xcd = bid % 8, k8 = bid / 8;
    const int lb = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k8;
    const int64_t wave0 = a.p0 + (int64_t)lb * kBlock + (threadIdx.x & ~(kWave - 1));
    if (__builtin_amdgcn_readfirstlane((int)(wave0 >= a.p1))) return;  // whole wave past the end
    const int64_t p = a.p0 + (int64_t)lb * kBlock + threadIdx.x;
    const bool valid = p < a.p1;
    const int64_t pp = valid ? p : a.p1 - 1;  // idle lanes shadow the last pivot

    const double xp = a.px[pp], yp = a.py[pp], zp = a.pz[pp];
    double th, sh = 0.0, ch = 0.0, phd = 0.0;
    float inv_sp = 0.0f, phf = 0.0f;
    // local north n and east e.  Off the poles e = n x r_p = (-y, x, 0) / |n| has no z
    // component for any pivot length; in the pole fallback (north along x, |y| < 1e-12) its z
    // component is y / |n|, and leaving that term out of the east coordinate turns the
    // bearing by less than 1e-12 |dz| / |d| (dz ~ |d|^2 / 2 there).  So e_z is never used.
    double nx, ny, nz, ex, ey;
    if constexpr (PLANAR) {
        // plane: strips of y, cells of x; angles from +y ("north") towards +x ("east")
        th = yp - a.py0;
        phd = (xp - a.px0) * a.psx;
        nx = 0.0; ny = 1.0; nz = 0.0;
        ex = 1.0; ey = 0.0;
    } else {
        const double sinth = sqrt(xp * xp + yp * yp);
        th = atan2(sinth, zp);
        double ph = atan2(yp, xp);
        if (ph < 0.0) ph += kTwoPi;
        sincos(0.5 * th, &sh, &ch);
        inv_sp = sinth > 0.0 ? (float)(1.0 / sinth) : INFINITY;
        phf = (float)ph;
        // local north and east
        nx = -zp * xp; ny = -zp * yp; nz = 1.0 - zp * zp;
        double nn = sqrt(nx * nx + ny * ny + nz * nz);
        if (nn < 1e-12) {
            nx = 1.0 - xp * xp; ny = -xp * yp; nz = -xp * zp;
            nn = sqrt(nx * nx + ny * ny + nz * nz);
        }
        nx /= nn; ny /= nn; nz /= nn;
        ex = ny * zp - nz * yp; ey = nz * xp - nx * zp;
    }

    // External pivots need not be unit vectors (the index's points are, to within the
    // windows' guards).  For a pivot of length rho = 1 + d and a unit neighbour at angle t,
    // the chord test reads d2 = d^2 + rho 4 hav(t), so the pair lies in [E_lo, E_hi) iff
    // hav(t) lies in [(E_lo - d^2) / 4 rho, (E_hi - d^2) / 4 rho): the wave's windows then
    // use the envelope of those bounds over its lanes (wave-uniform, per bin).
    double dmin = 0.0, dmax = 0.0;
    if constexpr (!PLANAR) {
        const double dp = sqrt(xp * xp + yp * yp + zp * zp) - 1.0;
        dmin = dp; dmax = dp;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            dmin = fmin(dmin, __shfl_xor(dmin, o, kWave));
            dmax = fmax(dmax, __shfl_xor(dmax, o, kWave));
        }
        dmin = uniform_f64(dmin);
        dmax = uniform_f64(dmax);
    }
    const bool rescale = __builtin_amdgcn_readfirstlane((int)!(dmin >= -kPivotNormTol && dmax <= kPivotNormTol));

    const int64_t col = p - a.p0;
    const int nb = a.nb;
    const bool unit_w = a.wdbl == nullptr;
    uint64_t my_pairs = 0;

    for (int bin = 0; bin < nb; ++bin) {
        const double elo = a.edges->e[bin], ehi = a.edges->e[bin + 1];
        double hav_out = a.edges->hav_out[bin + 1], hav_in = a.edges->hav_in[bin];
        double rad = a.edges->rad_out[bin + 1];
        if (rescale) {
            const double dsq = fmax(dmin * dmin, dmax * dmax);
            hav_out = 1.0 + fmin(dmin, 0.0) > 1e-3 ? fmin(hav_out / (1.0 + dmin) * (1.0 + 1e-15), 1.0 + 2e-9)
                                                   : 1.0 + 2e-9;
            hav_in = (hav_in - 0.25 * dsq) / (1.0 + fmax(dmax, 0.0)) * (1.0 - 1e-15) - 1e-300;
            rad = 2.0 * asin(fmin(1.0, sqrt(hav_out))) * (1.0 + 1e-9) + 1e-12;
            if (!(hav_in <= hav_out)) hav_in = -1.0;  // non-finite pivots: no inner exclusion
        }
        int klo = (int)floor((th - rad) * a.inv_h);
        int khi = (int)floor((th + rad) * a.inv_h);
        klo = max(klo, 0);
        khi = min(khi, a.nbands - 1);
        klo = __builtin_amdgcn_readfirstlane(wave_min(klo));
        khi = __builtin_amdgcn_readfirstlane(wave_max(khi));

        // SU_k = sum v U_k(cos phi) for k <= M, SV_k = sum v 2 sin(phi) U_k(cos phi) for k < M
        double SU[M + 1], SV[M + 1];
#pragma unroll
        for (int m = 0; m <= M; ++m) { SU[m] = 0.0; SV[m] = 0.0; }
        // wpend: the weight of the lane's previous pair, added at its next pair (or after the
        // bin), so that its load overlaps a candidate's work instead of stalling the pair that
        // requested it; the additions keep their order
        double Wb = 0.0, Qb = 0.0, wpend = 0.0;
        int cnt = 0;
        uint64_t hsum = 0;

        for (int k = klo; k <= khi; ++k) {
            const Band bd = a.bands[k];
            if (bd.npts == 0) continue;
            int s0, l0, s1, l1;
            if constexpr (PLANAR)
                planar_window(bd, a.cell_start, th, phd, a.psx, hav_out, hav_in, s0, l0, s1, l1);
            else
                band_window(bd, a.cell_start, th, sh, ch, inv_sp, phf, hav_out, hav_in, s0, l0, s1, l1);
            const int base = 2 * bd.pt_start;
            // the band's doubled records (wave-uniform base), walked by byte offset
            const __amdgpu_buffer_rsrc_t rband = buffer_view(a.rec + base, (uint32_t)bd.npts * 64u);
            // and its doubled weights (8 B per record: byte offset = record offset / 4)
            const __amdgpu_buffer_rsrc_t wband = buffer_view(unit_w ? nullptr : a.wdbl + base,
                                                             unit_w ? 0u : (uint32_t)bd.npts * 16u);
#pragma unroll
            for (int seg = 0; seg < 2; ++seg) {
                uint32_t off = (uint32_t)(seg == 0 ? s0 : s1) * 32u;
                const uint32_t oend = off + (uint32_t)(seg == 0 ? l0 : l1) * 32u;
                {
                    // one candidate at a time, its record requested one candidate ahead so
                    // that an L2 or HBM miss overlaps the previous candidate's work; two
                    // candidates per trip with two record registers in turn, so the record
                    // requested ahead needs no copy.  Past the window a request reads a
                    // record of the band that is never used (or, past the band, zeros from
                    // the buffer's range check).
                    auto cand = [&](const double4 &r, uint32_t o) __attribute__((always_inline)) {
                        const double dx = r.x - xp, dy = r.y - yp;
                        // on the plane both z are 0, and adding dz * dz = +0 to the
                        // non-negative sum changes nothing: the same d2 without that term
                        const double dz = PLANAR ? 0.0 : r.z - zp;
                        const double d2 = PLANAR ? dx * dx + dy * dy : (dx * dx + dy * dy) + dz * dz;
                        if (d2 >= elo && d2 < ehi) {
                            cnt += 1;
                            if constexpr (IDS) {
                                // record index from the byte offset, as an opaque shift so
                                // that the compiler keeps no second induction variable
                                uint32_t jo;
                                asm("v_lshrrev_b32 %0, 5, %1" : "=v"(jo) : "v"(o));
                                hsum += mix64((uint64_t)a.permdbl[base + (int)jo]);
                            }
                            if (!unit_w) {  // wave-uniform
                                Wb += wpend;
                                wpend = load_f64(wband, o >> 2);
                            }
                            const double v = r.w;
                            if constexpr (SELF) Qb = fma(v, v, Qb);
                            // plane: north +y, east +x, so the coordinates are dy and dx
                            const double u1 = PLANAR ? dy : fma(dx, nx, fma(dy, ny, dz * nz));
                            const double u2 = PLANAR ? dx : fma(dx, ex, dy * ey);
                            double tc, ts;  // 2 cos(phi), 2 sin(phi)
                            twice_unit_bearing(u1, u2, a.tiny, tc, ts);
                            SU[0] += v;
                            if constexpr (M >= 1) {
                                // one chain v U_k(cos phi): SU_k takes it, SV_k takes it
                                // times 2 sin(phi)
                                double ua = v, ub = tc * v;
                                SV[0] = fma(ts, v, SV[0]);
                                SU[1] += ub;
#pragma unroll
                                for (int k = 2; k <= M; ++k) {
                                    SV[k - 1] = fma(ts, ub, SV[k - 1]);
                                    const double uk = fma(tc, ub, -ua);
                                    SU[k] += uk;
                                    ua = ub; ub = uk;
                                }
                            }
                        }
                    };
                    double4 ra = load_record(rband, off < oend ? off : 0u);
                    for (; off < oend; off += 64u) {
                        const double4 rb = load_record(rband, off + 32u);
                        cand(ra, off);
                        if (off + 32u >= oend) break;
                        ra = load_record(rband, off + 64u);
                        cand(rb, off + 32u);
                    }
                }
            }
        }

        Wb += wpend;
        double self_t = 0.0;
        if (valid) {
            my_pairs += (uint64_t)cnt;
            if (unit_w) Wb = (double)cnt;
            double inv = 1.0;
            if (a.norm == Z3_NORM_BIN) inv = Wb > 0.0 ? 1.0 / Wb : 0.0;
            if constexpr (SELF) self_t = a.pv[p] * Qb * inv * inv;
            if (a.A) {
                // T_m = (U_m - U_{m-2}) / 2 (U_{-1} = 0) and sin(m phi) = sin(phi) U_{m-1}
                const double hinv = 0.5 * inv;
#pragma unroll
                for (int m = 0; m <= M; ++m) {
                    const double y = m >= 2 ? SU[m] - SU[m >= 2 ? m - 2 : 0] : SU[m];
                    const double re = m == 0 ? y * inv : y * hinv;
                    const double im = m == 0 ? 0.0 : -SV[m >= 1 ? m - 1 : 0] * hinv;
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
            const size_t ob = (size_t)bin * (size_t)a.ldA + col;
            if (a.W) a.W[ob] = Wb;
            if (a.counts) a.counts[ob] = cnt;
            if constexpr (IDS) a.idhash[ob] = hsum;
        }
        if constexpr (SELF) {
            const double t = wave_sum_f64(self_t);
            if ((threadIdx.x & (kWave - 1)) == 0)
                a.self_part[(size_t)((wave0 - a.p0) / kWave) * nb + bin] = t;
        }
    }

    if (a.pair_total) {
        const uint64_t tot = wave_sum_u64(valid ? my_pairs : 0);
        if ((threadIdx.x & (kWave - 1)) == 0 && tot) atomicAdd((unsigned long long *)a.pair_total, (unsigned long long)tot);
    }
}

// ---- many maps over one set of positions -------------------------------------------------
//
// Same decomposition (one lane per pivot, bins in order, band windows), but every lane
// carries K maps of a group of kMapGroup (K = 3 when the caller reads at most the first three,
// else 4): the pair test, the bearing and the unit chain U_k(cos phi) are computed once per
// pair, and each map adds v U_k and v 2 sin(phi) U_k with two FMAs per k (the epilogue forms
// the harmonics' sums as in k_multipoles).

struct MapArgs {
    const double *px, *py, *pz;   // index-order pivot positions
    const double4 *rec;           // doubled-band records (x, y, z used)
    const double *vgrp;           // [2n][kMapGroup] values of the map group
    const double *wdbl;           // doubled-band weights or null
    const int *cell_start;
    const Band *bands;
    int nbands;
    double inv_h;
    const EdgeTab *edges;
    int nb;
    int64_t p0, p1;
    void *A;                      // per map [m+1][2][nb][ldA], maps map_stride elements apart
    int64_t ldA;
    size_t map_stride;
    double *W;                    // [nb][ldA] W_{p,b} (shared by the maps), or null
    uint64_t *pair_total;
    int nblocks;
};

template <int M>
constexpr int maps_waves_per_eu()
{
    return M <= 6 ? 3 : 2;
}

template <int M, bool F32OUT, int K>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(maps_waves_per_eu<M>())))
void k_multipoles_maps(MapArgs a)
{
    static_assert(K == 3 || K == kMapGroup, "three or four maps per lane");
    const int nblk = a.nblocks;
    const int bid = blockIdx.x;
    const int per = nblk / 8, rem = nblk % 8;
    const int xcd = bid % 8, k8 = bid / 8;
    const int lb = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k8;
    const int64_t wave0 = a.p0 + (int64_t)lb * kBlock + (threadIdx.x & ~(kWave - 1));
    if (__builtin_amdgcn_readfirstlane((int)(wave0 >= a.p1))) return;
    const int64_t p = a.p0 + (int64_t)lb * kBlock + threadIdx.x;
    const bool valid = p < a.p1;
    const int64_t pp = valid ? p : a.p1 - 1;

    const double xp = a.px[pp], yp = a.py[pp], zp = a.pz[pp];
    const double sinth = sqrt(xp * xp + yp * yp);
    const double th = atan2(sinth, zp);
    double ph = atan2(yp, xp);
    if (ph < 0.0) ph += kTwoPi;
    double sh, ch;
    sincos(0.5 * th, &sh, &ch);
    const float inv_sp = sinth > 0.0 ? (float)(1.0 / sinth) : INFINITY;
    const float phf = (float)ph;
    double nx = -zp * xp, ny = -zp * yp, nz = 1.0 - zp * zp;
    double nn = sqrt(nx * nx + ny * ny + nz * nz);
    if (nn < 1e-12) {
        nx = 1.0 - xp * xp; ny = -xp * yp; nz = -xp * zp;
        nn = sqrt(nx * nx + ny * ny + nz * nz);
    }
    nx /= nn; ny /= nn; nz /= nn;
    // east without its z component, as in k_multipoles
    const double ex = ny * zp - nz * yp, ey = nz * xp - nx * zp;

    const int64_t col = p - a.p0;
    const int nb = a.nb;
    const bool unit_w = a.wdbl == nullptr;
    uint64_t my_pairs = 0;

    for (int bin = 0; bin < nb; ++bin) {
        const double elo = a.edges->e[bin], ehi = a.edges->e[bin + 1];
        const double hav_out = a.edges->hav_out[bin + 1], hav_in = a.edges->hav_in[bin];
        const double rad = a.edges->rad_out[bin + 1];
        int klo = (int)floor((th - rad) * a.inv_h);
        int khi = (int)floor((th + rad) * a.inv_h);
        klo = max(klo, 0);
        khi = min(khi, a.nbands - 1);
        klo = __builtin_amdgcn_readfirstlane(wave_min(klo));
        khi = __builtin_amdgcn_readfirstlane(wave_max(khi));

        // per map: SU_k = sum v U_k(cos phi), SV_k = sum v 2 sin(phi) U_k(cos phi), as in
        // k_multipoles, with one unit chain U_k shared by the maps
        double SU[K][M + 1], SV[K][M + 1];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int m = 0; m <= M; ++m) { SU[k][m] = 0.0; SV[k][m] = 0.0; }
        double Wb = 0.0;
        int cnt = 0;

        for (int kb = klo; kb <= khi; ++kb) {
            const Band bd = a.bands[kb];
            if (bd.npts == 0) continue;
            int s0, l0, s1, l1;
            band_window(bd, a.cell_start, th, sh, ch, inv_sp, phf, hav_out, hav_in, s0, l0, s1, l1);
            const int base = 2 * bd.pt_start;
#pragma unroll
            for (int seg = 0; seg < 2; ++seg) {
                int j = base + (seg == 0 ? s0 : s1);
                const int jend = j + (seg == 0 ? l0 : l1);
                for (; j < jend; ++j) {
                    const double4 r = a.rec[j];
                    const double dx = r.x - xp, dy = r.y - yp, dz = r.z - zp;
                    const double d2 = (dx * dx + dy * dy) + dz * dz;
                    if (d2 >= elo && d2 < ehi) {
                        cnt += 1;
                        if (!unit_w) Wb += a.wdbl[j];
                        const double4 vv = *reinterpret_cast<const double4 *>(a.vgrp + (size_t)j * kMapGroup);
                        double v[K];
                        v[0] = vv.x; v[1] = vv.y; v[2] = vv.z;
                        if constexpr (K == 4) v[3] = vv.w;
                        const double u1 = fma(dx, nx, fma(dy, ny, dz * nz));
                        const double u2 = fma(dx, ex, dy * ey);
                        double tc, ts;  // 2 cos(phi), 2 sin(phi)
                        twice_unit_bearing(u1, u2, kBearingTiny, tc, ts);
#pragma unroll
                        for (int k = 0; k < K; ++k) SU[k][0] += v[k];
                        if constexpr (M >= 1) {
                            double vs[K];
#pragma unroll
                            for (int k = 0; k < K; ++k) {
                                vs[k] = ts * v[k];
                                SV[k][0] += vs[k];
                                SU[k][1] = fma(v[k], tc, SU[k][1]);
                            }
                            double ua = 1.0, ub = tc;  // U_0, U_1
#pragma unroll
                            for (int m = 2; m <= M; ++m) {
#pragma unroll
                                for (int k = 0; k < K; ++k) SV[k][m - 1] = fma(vs[k], ub, SV[k][m - 1]);
                                const double um = fma(tc, ub, -ua);
#pragma unroll
                                for (int k = 0; k < K; ++k) SU[k][m] = fma(v[k], um, SU[k][m]);
                                ua = ub; ub = um;
                            }
                        }
                    }
                }
            }
        }

        if (valid) {
            my_pairs += (uint64_t)cnt;
            if (unit_w) Wb = (double)cnt;
            const double inv = Wb > 0.0 ? 1.0 / Wb : 0.0;
            const double hinv = 0.5 * inv;
            if (a.W) a.W[(size_t)bin * (size_t)a.ldA + col] = Wb;
#pragma unroll
            for (int k = 0; k < K; ++k) {
#pragma unroll
                for (int m = 0; m <= M; ++m) {
                    const double y = m >= 2 ? SU[k][m] - SU[k][m >= 2 ? m - 2 : 0] : SU[k][m];
                    const double re = m == 0 ? y * inv : y * hinv;
                    const double im = m == 0 ? 0.0 : -SV[k][m >= 1 ? m - 1 : 0] * hinv;
                    const size_t ore = k * a.map_stride + ((size_t)(2 * m) * nb + bin) * (size_t)a.ldA + col;
                    const size_t oim = k * a.map_stride + ((size_t)(2 * m + 1) * nb + bin) * (size_t)a.ldA + col;
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

    if (a.pair_total) {
        const uint64_t tot = wave_sum_u64(valid ? my_pairs : 0);
        if ((threadIdx.x & (kWave - 1)) == 0 && tot) atomicAdd((unsigned long long *)a.pair_total, (unsigned long long)tot);
    }
}

template <int M>
static void launch_maps_m(bool f32out, bool three, const MapArgs &a, hipStream_t s)
{
    dim3 grid(a.nblocks), block(kBlock);
    if (three) {
        if (f32out) hipLaunchKernelGGL((k_multipoles_maps<M, true, 3>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_multipoles_maps<M, false, 3>), grid, block, 0, s, a);
    } else {
        if (f32out) hipLaunchKernelGGL((k_multipoles_maps<M, true, kMapGroup>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_multipoles_maps<M, false, kMapGroup>), grid, block, 0, s, a);
    }
}

z3_status launch_multipoles_maps(const z3_index_s *idx, int group, int nslots, int m_max, int prec, int64_t p0,
                                 int64_t p1, void *A, int64_t ldA, size_t map_stride, double *W,
                                 uint64_t *pair_total, hipStream_t s)
{
    if (nslots < 1 || nslots > kMapGroup) return fail(Z3_ERR_INVALID_ARG, "map slots %d outside 1..%d", nslots, kMapGroup);
    int64_t nblk = (p1 - p0 + kBlock - 1) / kBlock;
    if (nblk > 0x7fffffff) return fail(Z3_ERR_OVERFLOW, "too many pivot blocks");
    MapArgs a;
    a.px = idx->d_x; a.py = idx->d_y; a.pz = idx->d_z;
    a.rec = idx->d_rec;
    a.vgrp = idx->d_vgrp + (size_t)group * 2 * idx->n * kMapGroup;
    a.wdbl = idx->unit_w ? nullptr : idx->d_wdbl;
    a.cell_start = idx->d_cell_start;
    a.bands = idx->d_bands;
    a.nbands = idx->nbands;
    a.inv_h = 1.0 / idx->band_h;
    a.edges = idx->d_edges;
    a.nb = idx->nbins;
    a.p0 = p0; a.p1 = p1;
    a.A = A; a.ldA = ldA; a.map_stride = map_stride;
    a.W = W;
    a.pair_total = pair_total;
    a.nblocks = (int)nblk;
    const bool f32 = prec == Z3_PREC_MIXED;
    hipEvent_t ev0;
    profile_begin(s, &ev0);
    switch (m_max) {
#define Z3_CASE(MM) case MM: launch_maps_m<MM>(f32, nslots <= 3, a, s); break;
        Z3_CASE(0) Z3_CASE(1) Z3_CASE(2) Z3_CASE(3) Z3_CASE(4) Z3_CASE(5) Z3_CASE(6) Z3_CASE(7)
        Z3_CASE(8) Z3_CASE(9) Z3_CASE(10) Z3_CASE(11) Z3_CASE(12) Z3_CASE(13) Z3_CASE(14)
        Z3_CASE(15) Z3_CASE(16)
#undef Z3_CASE
    default: return fail(Z3_ERR_UNSUPPORTED, "m_max=%d not compiled", m_max);
    }
    z3_status st = check_launch("k_multipoles_maps");
    profile_end(s, ev0);
    return st;
}

// The mixed path differs only in the output: FP32 multipoles for its split-FP32 contraction.
template <int M, bool PLANAR>
static void launch_mp(bool f32out, bool ids, bool self, const MultArgs &a, hipStream_t s)
{
    dim3 grid(a.nblocks), block(kBlock);
    if (f32out) {
        if (ids) hipLaunchKernelGGL((k_multipoles<M, true, true, false, PLANAR>), grid, block, 0, s, a);
        else if (self) hipLaunchKernelGGL((k_multipoles<M, true, false, true, PLANAR>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_multipoles<M, true, false, false, PLANAR>), grid, block, 0, s, a);
    } else {
        if (ids) hipLaunchKernelGGL((k_multipoles<M, false, true, false, PLANAR>), grid, block, 0, s, a);
        else if (self) hipLaunchKernelGGL((k_multipoles<M, false, false, true, PLANAR>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_multipoles<M, false, false, false, PLANAR>), grid, block, 0, s, a);
    }
}

template <int M>
static void launch_m(bool planar, bool mixed, bool ids, bool self, const MultArgs &a, hipStream_t s)
{
    if (planar) launch_mp<M, true>(mixed, ids, self, a, s);
    else launch_mp<M, false>(mixed, ids, self, a, s);
}

z3_status launch_multipoles(const z3_index_s *idx, Pivots piv, int map, int m_max, int prec, int norm,
                            int64_t p0, int64_t p1, void *A, int64_t ldA, double *W,
                            int64_t *counts, uint64_t *idhash, uint64_t *pair_total, hipStream_t s,
                            const double *self_pv, double *self_part)
{
    int64_t nblk = (p1 - p0 + kBlock - 1) / kBlock;
    if (nblk > 0x7fffffff) return fail(Z3_ERR_OVERFLOW, "too many pivot blocks");
    if ((self_part != nullptr) != (self_pv != nullptr) || (self_part && idhash))
        return fail(Z3_ERR_INVALID_ARG, "k_multipoles: the self-pair sums need pivot values and no fingerprints");
    MultArgs a;
    a.px = piv.x; a.py = piv.y; a.pz = piv.z;
    a.rec = idx->d_rec + (size_t)map * 2 * idx->n;
    a.wdbl = idx->unit_w ? nullptr : idx->d_wdbl;
    a.permdbl = idx->d_permdbl;
    a.cell_start = idx->d_cell_start;
    a.bands = idx->d_bands;
    a.nbands = idx->nbands;
    a.inv_h = 1.0 / idx->band_h;
    a.edges = idx->d_edges;
    a.nb = idx->nbins;
    a.p0 = p0; a.p1 = p1;
    a.norm = norm;
    a.A = A; a.ldA = ldA;
    a.W = W; a.counts = counts; a.idhash = idhash; a.pair_total = pair_total;
    a.pv = self_pv; a.self_part = self_part;
    a.px0 = idx->plane_x0; a.py0 = idx->plane_y0; a.psx = idx->plane_sx;
    a.tiny = kBearingTiny;
    a.nblocks = (int)nblk;
    const bool mixed = prec == Z3_PREC_MIXED, ids = idhash != nullptr, self = self_part != nullptr;
    hipEvent_t ev0;
    profile_begin(s, &ev0);
    switch (m_max) {
#define Z3_CASE(MM) case MM: launch_m<MM>(idx->planar, mixed, ids, self, a, s); break;
        Z3_CASE(0) Z3_CASE(1) Z3_CASE(2) Z3_CASE(3) Z3_CASE(4) Z3_CASE(5) Z3_CASE(6) Z3_CASE(7)
        Z3_CASE(8) Z3_CASE(9) Z3_CASE(10) Z3_CASE(11) Z3_CASE(12) Z3_CASE(13) Z3_CASE(14)
        Z3_CASE(15) Z3_CASE(16)
#undef Z3_CASE
    default: return fail(Z3_ERR_UNSUPPORTED, "m_max=%d not compiled", m_max);
    }
    z3_status st = check_launch("k_multipoles");
    profile_end(s, ev0);
    return st;
}

}  // namespace z3
