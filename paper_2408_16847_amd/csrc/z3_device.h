// Device helpers shared by the multipole, many-map and adjoint kernels (internal).
#pragma once

#include "z3_internal.h"

namespace z3 {

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// A wave-uniform double moved to scalar registers (the value of the first active lane).
__device__ __forceinline__ double uniform_f64(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __builtin_bit_cast(double, (uint64_t)hi << 32 | lo);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
    unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
    // two 32-bit halves, carried through a 64-bit sum at every step
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned olo = __shfl_xor(lo, o, 64), ohi = __shfl_xor(hi, o, 64);
        uint64_t s = ((uint64_t)hi << 32 | lo) + ((uint64_t)ohi << 32 | olo);
        lo = (unsigned)s;
        hi = (unsigned)(s >> 32);
    }
    return (uint64_t)hi << 32 | lo;
}

// Butterfly sum over the wave; the order of the additions is fixed, so the result is
// reproducible from run to run.
__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Buffer view of one band's doubled records: a gfx9 buffer resource on a wave-uniform
// base, addressed by 32-bit per-lane byte offsets (one add and one compare per loop step
// instead of 64-bit address arithmetic).  Loads past `bytes` return zeros.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_view(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

// One FP64 value at byte offset `off` of a buffer view (0 past its range).
__device__ __forceinline__ double load_f64(__amdgpu_buffer_rsrc_t v, uint32_t off)
{
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 a = __builtin_amdgcn_raw_buffer_load_b64(v, off, 0, 0);
    return __builtin_bit_cast(double, (uint64_t)a.x | (uint64_t)a.y << 32);
}

__device__ __forceinline__ double4 load_record(__amdgpu_buffer_rsrc_t v, uint32_t off)
{
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    const u4 a = __builtin_amdgcn_raw_buffer_load_b128(v, off, 0, 0);
    const u4 b = __builtin_amdgcn_raw_buffer_load_b128(v, off + 16u, 0, 0);
    double4 r;
    r.x = __builtin_bit_cast(double, (uint64_t)a.x | (uint64_t)a.y << 32);
    r.y = __builtin_bit_cast(double, (uint64_t)a.z | (uint64_t)a.w << 32);
    r.z = __builtin_bit_cast(double, (uint64_t)b.x | (uint64_t)b.y << 32);
    r.w = __builtin_bit_cast(double, (uint64_t)b.z | (uint64_t)b.w << 32);
    return r;
}

__device__ __forceinline__ uint64_t mix64(uint64_t v)
{  // SplitMix64 finaliser (Steele, Lea & Flood 2014)
    v += 0x9E3779B97F4A7C15ull;
    v = (v ^ (v >> 30)) * 0xBF58476D1CE4E5B9ull;
    v = (v ^ (v >> 27)) * 0x94D049BB133111EBull;
    return v ^ (v >> 31);
}

// Logical cell range [ca, cb] of a band (indices may run one band-length below 0 or
// above ncell to express wrap-around) -> start (in [0, npts)) and length in points.
__device__ __forceinline__ void cells_to_points(const Band &bd, const int *cell_start, int ca, int cb,
                                                int &s, int &len)
{
    if (cb < ca) {
        s = 0;
        len = 0;
        return;
    }
    const int C = bd.ncell, np = bd.npts;
    // windows span at most one band length around [0, C); the clamps only matter for
    // non-finite inputs and keep every index inside the band regardless.  With
    // ca in [-C, 2C) and cb + 1 in [-C + 1, 2C], the band-length quotients are -1, 0 or 1.
    ca = max(ca, -C);
    cb = min(cb, 2 * C - 1);
    const int q0 = ca < 0 ? -1 : (ca >= C ? 1 : 0), r0 = ca - q0 * C;
    const int q1 = cb + 1 < 0 ? -1 : (cb + 1 >= C ? 1 : 0), r1 = cb + 1 - q1 * C;
    const int st = cell_start[bd.cell_off + r0] - bd.pt_start + q0 * np;
    const int en = cell_start[bd.cell_off + r1] - bd.pt_start + q1 * np;
    len = min(max(en - st, 0), np);
    s = st < 0 ? st + np : (st >= np ? st - np : st);
    s = min(max(s, 0), np - 1);
}

// Longitude window(s) of band `bd` that can hold points at angular distance in
// [R_in, R_out) of the pivot, with hav(R) = E/4 (hav_in, hav_out already carry their
// rounding guards).  Spherical law of haversines, for a point at colatitude t in the
// band and longitude offset dphi:
//     hav(d) = hav(t - th_p) + sin(th_p) sin(t) hav(dphi)
// so d < R_out needs hav(dphi) < (hav_out - min hav(t - th_p)) / (sin th_p * min sin t),
// and d >= R_in needs hav(dphi) >= (hav_in - max hav(t - th_p)) / (sin th_p * max sin t).
__device__ __forceinline__ void band_window(const Band &bd, const int *cell_start, double th, double sh,
                                            double ch, float inv_sp, float phf, double hav_out,
                                            double hav_in, int &s0, int &l0, int &s1, int &l1)
{
    s0 = l0 = s1 = l1 = 0;
    const double dlo = bd.sh_lo * ch - bd.ch_lo * sh;  // sin((th_lo - th_p) / 2)
    const double dhi = bd.sh_hi * ch - bd.ch_hi * sh;  // sin((th_hi - th_p) / 2)
    const double hlo = dlo * dlo, hhi = dhi * dhi;
    const double hmin = th < bd.th_lo ? hlo : (th > bd.th_hi ? hhi : 0.0);
    const double hmax = fmax(hlo, hhi);
    const double num_out = hav_out - hmin;
    if (!(num_out > 0.0)) return;  // the band lies entirely beyond R_out
    const double num_in = hav_in - hmax;
    const int C = bd.ncell;
    const float cpr = bd.cells_per_rad;

    // The half-widths asin(sqrt(q)) are bounded rather than evaluated: with a = asin(x),
    // x <= a <= tan(a) = x / sqrt(1 - x^2), so sqrt(q) bounds the excluded arc from below
    // and sqrt(q / (1 - q)) the window from above (relative excess ~a^2 / 3, a few extra
    // candidates that the d2 test rejects).  Hardware square root and reciprocal square
    // root (~1 ulp) sit far inside the guard factors.
    const float q_out = (float)num_out * inv_sp * bd.inv_smin * (1.0f + 1e-5f);
    bool full = !(q_out < 1.0f);
    float dout = 0.0f;
    if (!full) {
        const float t = __builtin_amdgcn_sqrtf(q_out) * __builtin_amdgcn_rsqf(1.0f - q_out);
        dout = 2.0f * t * (1.0f + 4e-6f) + 4e-6f;
        full = !(dout < 3.14159265f);
    }
    bool excl = false;
    float din = 0.0f;
    if (num_in > 0.0) {
        const float q_in = (float)num_in * inv_sp * bd.inv_smax * (1.0f - 1e-5f);
        if (!(q_in < 1.0f)) return;  // the whole band lies inside R_in
        din = 2.0f * __builtin_amdgcn_sqrtf(q_in) * (1.0f - 4e-6f) - 4e-6f;
        excl = din > 0.0f;
    }
    // cells entirely inside the excluded arc (phf - din, phf + din)
    int es = 0, ee = -1;
    const float lim = 2.0f * (float)C;  // window bounds stay within +-2 band lengths
    if (excl) {
        es = (int)fminf(fmaxf(ceilf((phf - din) * cpr), -lim), lim);
        ee = (int)fminf(fmaxf(floorf((phf + din) * cpr), -lim), lim) - 1;
    }
    int ca0 = 0, cb0 = -1, ca1 = 0, cb1 = -1;
    if (!full) {
        const int clo = (int)fminf(fmaxf(floorf((phf - dout) * cpr), -lim), lim);
        const int chi = (int)fminf(fmaxf(floorf((phf + dout) * cpr), -lim), lim);
        if (chi - clo + 1 >= C) {
            full = true;
        } else {
            if (excl) {
                es = max(es, clo);
                ee = min(ee, chi);
            }
            if (excl && es <= ee) {
                ca0 = clo; cb0 = es - 1;
                ca1 = ee + 1; cb1 = chi;
            } else {
                ca0 = clo; cb0 = chi;
            }
        }
    }
    if (full) {
        if (excl && es <= ee) {
            if (ee - es + 1 >= C) return;
            ca0 = ee + 1; cb0 = es - 1 + C;
        } else {
            ca0 = 0; cb0 = C - 1;
        }
        ca1 = 0; cb1 = -1;
    }
    cells_to_points(bd, cell_start, ca0, cb0, s0, l0);
    cells_to_points(bd, cell_start, ca1, cb1, s1, l1);
}

// Window(s) of a strip for pivots on a plane: the strip's points have y - y0 in
// [th_lo, th_hi] and cell coordinate (x - x0) sx; a point at distance in [R_in, R_out)
// of the pivot (y - y0 = yrel, cell coordinate phd) has |dx| < sqrt(R_out^2 - dy_min^2)
// and, when the strip lies within R_in in y, |dx| >= sqrt(R_in^2 - dy_max^2).  r2_out and
// r2_in are the guarded squared radii; the cells entirely inside the inner gap are
// skipped, which leaves up to two ranges.  Bounds in FP64, clamped to the strip.
__device__ __forceinline__ void planar_window(const Band &bd, const int *cell_start, double yrel, double phd,
                                              double sx, double r2_out, double r2_in, int &s0, int &l0, int &s1,
                                              int &l1)
{
    s0 = l0 = s1 = l1 = 0;
    const double dlo = bd.th_lo - yrel, dhi = bd.th_hi - yrel;
    const double dymin = (dlo <= 0.0 && dhi >= 0.0) ? 0.0 : fmin(fabs(dlo), fabs(dhi));
    const double dymax = fmax(fabs(dlo), fabs(dhi));
    const double q_out = r2_out - dymin * dymin;
    if (!(q_out > 0.0)) return;  // the strip lies entirely beyond R_out
    const int C = bd.ncell;
    const double cpr = (double)C / kTwoPi;  // as in the cell assignment
    const double lim = (double)(C - 1);
    const double dout = sqrt(q_out) * (1.0 + 1e-9) * sx + 1e-12;
    const int clo = (int)fmin(fmax(floor((phd - dout) * cpr), 0.0), lim);
    const int chi = (int)fmin(fmax(floor((phd + dout) * cpr), 0.0), lim);
    int es = 0, ee = -1;
    const double q_in = r2_in - dymax * dymax;
    if (q_in > 0.0) {
        const double din = sqrt(q_in) * (1.0 - 1e-9) * sx - 1e-12;
        if (din > 0.0) {
            // cells [es, ee] lie entirely inside (phd - din, phd + din)
            es = (int)fmin(fmax(ceil((phd - din) * cpr), -1.0), lim + 1.0);
            ee = (int)fmin(fmax(floor((phd + din) * cpr), 0.0), lim + 1.0) - 1;
            es = max(es, clo);
            ee = min(ee, chi);
        }
    }
    if (es <= ee) {
        cells_to_points(bd, cell_start, clo, es - 1, s0, l0);
        cells_to_points(bd, cell_start, ee + 1, chi, s1, l1);
    } else {
        cells_to_points(bd, cell_start, clo, chi, s0, l0);
    }
}

// Unit-length bearing (c, s) = (u1, u2) / |u| with FP64 accuracy: FP32 reciprocal
// square root refined by one FP64 Newton step (relative error ~1e-14).  For every pair in
// range |u|^2 >= E_0 (1 - E_nb / 4) > 0; the addend below only matters for |u| = 0.
__device__ __forceinline__ void unit_bearing(double u1, double u2, double &c, double &s)
{
    // the tiny addend keeps q > 0 (coincident points) at the cost of no instruction: it is
    // below the rounding of u2^2 for every pair in range
    const double q = fma(u1, u1, fma(u2, u2, 1e-37));
    const double r0 = (double)__builtin_amdgcn_rsqf((float)q);
    const double e = fma(-q * r0, r0, 1.0);  // 1 - q r0^2
    const double r = fma(0.5 * e, r0, r0);
    c = u1 * r;
    s = u2 * r;
}

// (2 cos phi, 2 sin phi) of the bearing: unit_bearing's refinement with the factor 2 folded
// into the refined reciprocal length (2 r = 2 r0 + e r0).  `tiny` is unit_bearing's addend
// (kBearingTiny); a kernel that takes it as an argument holds it in scalar registers, so
// the first FMA reads it there instead of from a vector register copied per pair.
constexpr double kBearingTiny = 1e-37;
__device__ __forceinline__ void twice_unit_bearing(double u1, double u2, double tiny, double &c2, double &s2)
{
    const double q = fma(u1, u1, fma(u2, u2, tiny));
    const double r0 = (double)__builtin_amdgcn_rsqf((float)q);
    const double e = fma(-q * r0, r0, 1.0);
    const double r2 = fma(e, r0, r0 + r0);
    c2 = u1 * r2;
    s2 = u2 * r2;
}

// XCD-aware block order: the hardware hands consecutive block ids to the 8 XCDs in turn;
// this bijection gives each XCD a contiguous run of logical tiles, so the neighbour data
// of adjacent pivots stays in one L2.
__device__ __forceinline__ int xcd_block(int bid, int nblk)
{
    const int per = nblk / 8, rem = nblk % 8;
    const int xcd = bid % 8, k8 = bid / 8;
    return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + k8;
}

// Everything a lane needs about its pivot: position, colatitude and longitude (for the
// band windows), and the local north / east unit vectors of the bearing.
struct PivotFrame {
    double xp, yp, zp;
    double th, sh, ch;     // colatitude and sin/cos of its half
    float inv_sp, phf;     // 1 / sin(colatitude), longitude in [0, 2 pi)
    double nx, ny, nz;     // local north
    double ex, ey;         // local east; its z component is left out (see pivot_frame)
};

__device__ __forceinline__ PivotFrame pivot_frame(double xp, double yp, double zp)
{
    PivotFrame f;
    f.xp = xp; f.yp = yp; f.zp = zp;
    const double sinth = sqrt(xp * xp + yp * yp);
    f.th = atan2(sinth, zp);
    double ph = atan2(yp, xp);
    if (ph < 0.0) ph += kTwoPi;
    sincos(0.5 * f.th, &f.sh, &f.ch);
    f.inv_sp = sinth > 0.0 ? (float)(1.0 / sinth) : INFINITY;
    f.phf = (float)ph;
    double nx = -zp * xp, ny = -zp * yp, nz = 1.0 - zp * zp;
    double nn = sqrt(nx * nx + ny * ny + nz * nz);
    if (nn < 1e-12) {  // at a pole: measure from the x axis instead
        nx = 1.0 - xp * xp; ny = -xp * yp; nz = -xp * zp;
        nn = sqrt(nx * nx + ny * ny + nz * nz);
    }
    f.nx = nx / nn; f.ny = ny / nn; f.nz = nz / nn;
    // east = north x r_p.  Off the poles that is (-y, x, 0) / |n|, with no z component for
    // any pivot length; in the pole fallback its z component is y / |n| with |y| < 1e-12, and
    // leaving it out of the east coordinate turns the bearing by less than 1e-12 |dz| / |d|.
    f.ex = f.ny * zp - f.nz * yp;
    f.ey = f.nz * xp - f.nx * zp;
    return f;
}

// Bands that can hold neighbours within angular radius `rad` of any lane's pivot
// (uniform across the wave).
__device__ __forceinline__ void band_range(double th, double rad, double inv_h, int nbands, int &klo, int &khi)
{
    int lo = (int)floor((th - rad) * inv_h);
    int hi = (int)floor((th + rad) * inv_h);
    lo = max(lo, 0);
    hi = min(hi, nbands - 1);
    klo = __builtin_amdgcn_readfirstlane(wave_min(lo));
    khi = __builtin_amdgcn_readfirstlane(wave_max(hi));
}

}  // namespace z3
