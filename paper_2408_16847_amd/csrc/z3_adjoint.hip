// Adjoint of the estimator with respect to the field values (vector-Jacobian product).
//
// For a real loss L of zeta and G_m(b1, b2) = dL/dRe zeta + i dL/dIm zeta, with
// v_p = w_p x_p and X_p(b) = sum_{j in b(p)} c_pj x_j, c_pj = w_j exp(-i m phi_pj) / W_{p,b}
// (eqs. Xm.binned and zetamEst), the gradient of L(scale * sum_p v_p X_p X_p^H) is
//
//   dL/dx_k = scale * w_k Re sum_m sum_{b1 b2} conj(G(b1,b2)) X_k(b1) conj(X_k(b2))       (pivot)
//           + scale * sum_{p: k in bin a of p} v_p Re sum_m c_pk D_p(a),                     (neighbour)
//   D_p(a)  = sum_b (conj(G(a,b)) + G(b,a)) conj(X_p(b)).
//
// Per pivot chunk: (1) the multipole kernel recomputes X_p and W_{p,b} (nothing is kept
// between chunks); (2) k_adjoint_prep forms D_p(a) / W_{p,a} and adds the pivot term
// (grid y: the maps of the pass);
// (3) k_adjoint_scatter walks the same bin/band windows as the forward kernel, rebuilds
// the harmonics per pair (as second-kind Chebyshev polynomials of cos phi) and adds the neighbour term to the neighbour's gradient
// with an FP64 atomic (index order; permuted to catalogue order at the end).  The atomics
// make the last bits of the gradient depend on scheduling.
#include "z3_internal.h"
#include "z3_device.h"

namespace z3 {

struct PrepArgs {
    const double *A;   // [m+1][2][nb][P] X_p (normalised)
    const double *W;   // [nb][P]
    const double *G;   // [m+1][nb][nb][2]
    const double *v;   // [P] pivot w x
    const double *w;   // [P] pivot weights
    double *D;         // [m+1][2][nb][P] D_p(a) / W_{p,a}
    double *grad;      // index-order gradient, pivot term added for p in [p0, p0 + P)
    int64_t P;
    int nb, M;
    double scale;
    // map blockIdx.y: A and D advance by ad_stride, G by g_stride, v and grad by n_stride
    size_t ad_stride, g_stride, n_stride;
};

// One thread per (pivot, map); for each m the block first forms
//     H(a, b) = conj(G(a, b)) + G(b, a)
// in LDS (G is shared by the block's map), then every thread keeps its X(b) in registers:
//     D(a) = sum_b H(a, b) conj(X(b)),
// and the pivot term is Re sum_a X(a) E(a) = Re sum_a X(a) D(a) / 2, since
// sum_a X(a) F(a) = conj(sum_a X(a) E(a)) (swap a and b).  NBT bounds nb (registers).
template <int NBT>
__global__ __launch_bounds__(256) void k_adjoint_prep(PrepArgs a)
{
    __shared__ double2 sH[NBT * NBT];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = p < a.P;
    const size_t mp = blockIdx.y;
    const double *A = a.A + mp * a.ad_stride;
    double *D = a.D + mp * a.ad_stride;
    const double *G = a.G + mp * a.g_stride;
    const int nb = a.nb;
    const size_t P = (size_t)a.P;
    const size_t pc = act ? (size_t)p : 0;
    double piv = 0.0;
    // up to 16 bins the a-loop is unrolled too: 1 / W_{p,a} is loaded once, and X(a) comes
    // from the registers instead of a second load
    constexpr bool UNROLL_A = NBT <= 16;
    double inv_w[UNROLL_A ? NBT : 1];
    if constexpr (UNROLL_A) {
#pragma unroll
        for (int ai = 0; ai < NBT; ++ai) {
            const double wa = ai < nb ? a.W[(size_t)ai * P + pc] : 0.0;
            inv_w[ai] = wa > 0.0 ? 1.0 / wa : 0.0;
        }
    }
    for (int m = 0; m <= a.M; ++m) {
        __syncthreads();  // the previous m's H is consumed
        const double *g = G + (size_t)m * nb * nb * 2;
        for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
            const int ai = e / nb, b = e - ai * nb;
            const double gr = g[((size_t)ai * nb + b) * 2], gi = g[((size_t)ai * nb + b) * 2 + 1];
            const double tr = g[((size_t)b * nb + ai) * 2], ti = g[((size_t)b * nb + ai) * 2 + 1];
            sH[ai * NBT + b] = make_double2(gr + tr, ti - gi);
        }
        __syncthreads();
        if (!act) continue;
        const double *xr = A + (size_t)(2 * m) * nb * P + pc;
        const double *xi = A + (size_t)(2 * m + 1) * nb * P + pc;
        double ur[NBT], ui[NBT];  // conj(X(b))
#pragma unroll
        for (int b = 0; b < NBT; ++b) {
            ur[b] = b < nb ? xr[(size_t)b * P] : 0.0;
            ui[b] = b < nb ? -xi[(size_t)b * P] : 0.0;
        }
        if constexpr (UNROLL_A) {
#pragma unroll
            for (int ai = 0; ai < NBT; ++ai) {
                if (ai >= nb) continue;  // uniform
                double dr = 0.0, di = 0.0;
#pragma unroll
                for (int b = 0; b < NBT; ++b) {
                    if (b < nb) {
                        const double2 h = sH[ai * NBT + b];
                        dr = fma(h.x, ur[b], fma(-h.y, ui[b], dr));
                        di = fma(h.x, ui[b], fma(h.y, ur[b], di));
                    }
                }
                piv += 0.5 * (ur[ai] * dr + ui[ai] * di);  // Re(X(a) D(a)) / 2, X = (ur, -ui)
                D[((size_t)(2 * m) * nb + ai) * P + pc] = dr * inv_w[ai];
                D[((size_t)(2 * m + 1) * nb + ai) * P + pc] = di * inv_w[ai];
            }
            continue;
        }
        for (int ai = 0; ai < nb; ++ai) {
            double dr = 0.0, di = 0.0;
#pragma unroll
            for (int b = 0; b < NBT; ++b) {
                if (b < nb) {  // uniform
                    const double2 h = sH[ai * NBT + b];
                    dr = fma(h.x, ur[b], fma(-h.y, ui[b], dr));
                    di = fma(h.x, ui[b], fma(h.y, ur[b], di));
                }
            }
            const double x_r = xr[(size_t)ai * P], x_i = xi[(size_t)ai * P];
            piv += 0.5 * (x_r * dr - x_i * di);
            const double wa = a.W[(size_t)ai * P + pc];
            const double inv = wa > 0.0 ? 1.0 / wa : 0.0;
            D[((size_t)(2 * m) * nb + ai) * P + pc] = dr * inv;
            D[((size_t)(2 * m + 1) * nb + ai) * P + pc] = di * inv;
        }
    }
    if (act) a.grad[mp * a.n_stride + pc] += a.scale * a.w[pc] * piv;
}

// The same for any nb: X(b) read from memory in the inner loop.
__global__ __launch_bounds__(256) void k_adjoint_prep_any(PrepArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    const size_t mp = blockIdx.y;
    const double *A = a.A + mp * a.ad_stride;
    double *D = a.D + mp * a.ad_stride;
    const double *G = a.G + mp * a.g_stride;
    const int nb = a.nb;
    const size_t P = (size_t)a.P;
    double piv = 0.0;
    for (int m = 0; m <= a.M; ++m) {
        const double *xr = A + (size_t)(2 * m) * nb * P + p;
        const double *xi = A + (size_t)(2 * m + 1) * nb * P + p;
        const double *g = G + (size_t)m * nb * nb * 2;
        for (int ai = 0; ai < nb; ++ai) {
            double dr = 0.0, di = 0.0;
            for (int b = 0; b < nb; ++b) {
                const double ur = xr[(size_t)b * P], ui = -xi[(size_t)b * P];
                const double hr = g[((size_t)ai * nb + b) * 2] + g[((size_t)b * nb + ai) * 2];
                const double hi = g[((size_t)b * nb + ai) * 2 + 1] - g[((size_t)ai * nb + b) * 2 + 1];
                dr = fma(hr, ur, fma(-hi, ui, dr));
                di = fma(hr, ui, fma(hi, ur, di));
            }
            const double x_r = xr[(size_t)ai * P], x_i = xi[(size_t)ai * P];
            piv += 0.5 * (x_r * dr - x_i * di);
            const double wa = a.W[(size_t)ai * P + p];
            const double inv = wa > 0.0 ? 1.0 / wa : 0.0;
            D[((size_t)(2 * m) * nb + ai) * P + p] = dr * inv;
            D[((size_t)(2 * m + 1) * nb + ai) * P + p] = di * inv;
        }
    }
    a.grad[mp * a.n_stride + p] += a.scale * a.w[p] * piv;
}

struct ScatterArgs {
    const double *px, *py, *pz;   // index-order pivot positions
    const double *pv;             // index-order w x of the map (pivot values)
    const double4 *rec;           // doubled-band records
    const double *wdbl;           // doubled-band weights or null
    const int *cell_start;
    const Band *bands;
    int nbands;
    double inv_h;
    const EdgeTab *edges;
    int nb;
    int64_t p0, p1;
    const double *D;              // [m+1][2][nb][ldD] for pivots [p0, p1)
    int64_t ldD;
    double *grad;                 // index-order gradient
    double scale;
    int nblocks;
    // map blockIdx.y: pv and grad advance by n_stride, rec by rec_stride, D by d_stride
    size_t n_stride, rec_stride, d_stride;
    double px0, py0, psx;         // plane: origin and cell-coordinate scale
};

// Pivot on a plane: strip coordinate y - y0 in place of the colatitude, fixed frame
// (angles from +y towards +x); the longitude fields are unused.
__device__ __forceinline__ PivotFrame plane_frame(double xp, double yp, double zp, double y0)
{
    PivotFrame f;
    f.xp = xp; f.yp = yp; f.zp = zp;
    f.th = yp - y0;
    f.sh = 0.0; f.ch = 0.0; f.inv_sp = 0.0f; f.phf = 0.0f;
    f.nx = 0.0; f.ny = 1.0; f.nz = 0.0;
    f.ex = 1.0; f.ey = 0.0;
    return f;
}

// K maps per lane share each pair's geometry and harmonics; their D coefficients take
// 2 (M + 1) K registers, so the occupancy target drops with K.
template <int M, int K>
constexpr int adjoint_waves_per_eu()
{
    return K == 1 ? (M <= 10 ? 4 : (M <= 13 ? 3 : 2)) : (K == 2 && M <= 10 ? 3 : 2);
}

// Per-wave LDS slice that gathers a window's contributions before they go to HBM: the
// lanes of a wave walk overlapping ranges of the same band, so one window's pairs touch
// only ~(window + 64) distinct neighbours.  kAggSlots doubles per wave, split among the K
// maps.
constexpr int kAggSlots = 1024;

template <int M, int K, bool PLANAR = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(adjoint_waves_per_eu<M, K>())))
void k_adjoint_scatter(ScatterArgs a)
{
    constexpr int SLOTS = kAggSlots / K;
    __shared__ double agg_all[kBlock / kWave][K][SLOTS];
    double(*agg)[SLOTS] = agg_all[threadIdx.x / kWave];
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int k = 0; k < K; ++k)
        for (int e = lane; e < SLOTS; e += kWave) agg[k][e] = 0.0;
    const int lb = xcd_block(blockIdx.x, a.nblocks);
    const int64_t wave0 = a.p0 + (int64_t)lb * kBlock + (threadIdx.x & ~(kWave - 1));
    if (__builtin_amdgcn_readfirstlane((int)(wave0 >= a.p1))) return;
    const int64_t p = a.p0 + (int64_t)lb * kBlock + threadIdx.x;
    const bool valid = p < a.p1;
    const int64_t pp = valid ? p : a.p1 - 1;
    const size_t mp0 = (size_t)blockIdx.y * K;  // first map of this block
    a.rec += mp0 * a.rec_stride;  // positions (the same for every map)
    const PivotFrame f = PLANAR ? plane_frame(a.px[pp], a.py[pp], a.pz[pp], a.py0)
                                : pivot_frame(a.px[pp], a.py[pp], a.pz[pp]);
    const double phd = PLANAR ? (a.px[pp] - a.px0) * a.psx : 0.0;
    double vp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) vp[k] = valid ? a.scale * a.pv[(mp0 + k) * a.n_stride + pp] : 0.0;  // idle lanes add nothing
    const int64_t col = pp - a.p0;
    const int nb = a.nb;
    const bool unit_w = a.wdbl == nullptr;

    for (int bin = 0; bin < nb; ++bin) {
        const double elo = a.edges->e[bin], ehi = a.edges->e[bin + 1];
        const double hav_out = a.edges->hav_out[bin + 1], hav_in = a.edges->hav_in[bin];
        int klo, khi;
        band_range(f.th, a.edges->rad_out[bin + 1], a.inv_h, a.nbands, klo, khi);
        // sum_m cos(m phi) Dr_m + sin(m phi) Di_m rewritten on the second-kind polynomials of
        // c = cos phi (T_m = (U_m - U_{m-2}) / 2, sin(m phi) = sin(phi) U_{m-1}):
        //   sum_k U_k(c) (Al_k + 2 sin(phi) Bt_k),
        //   Al_0 = Dr_0 - Dr_2 / 2,  Al_k = (Dr_k - Dr_{k+2}) / 2,  Bt_k = Di_{k+1} / 2,
        // so that each pair runs one unit chain U_k and two FMAs per k and map.
        double Al[K][M + 1], Bt[K][M + 1];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double *Dk = a.D + (mp0 + k) * a.d_stride;
            double Dr[M + 1], Di[M + 1];
#pragma unroll
            for (int m = 0; m <= M; ++m) {
                Dr[m] = vp[k] * Dk[((size_t)(2 * m) * nb + bin) * (size_t)a.ldD + col];
                Di[m] = vp[k] * Dk[((size_t)(2 * m + 1) * nb + bin) * (size_t)a.ldD + col];
            }
#pragma unroll
            for (int m = 0; m <= M; ++m) {
                const double hi = m + 2 <= M ? 0.5 * Dr[m + 2 <= M ? m + 2 : 0] : 0.0;
                Al[k][m] = (m == 0 ? Dr[0] : 0.5 * Dr[m]) - hi;
                Bt[k][m] = m < M ? 0.5 * Di[m < M ? m + 1 : 0] : 0.0;
            }
        }
        for (int kb = klo; kb <= khi; ++kb) {
            const Band bd = a.bands[kb];
            if (bd.npts == 0) continue;
            int s0, l0, s1, l1;
            if constexpr (PLANAR)
                planar_window(bd, a.cell_start, f.th, phd, a.psx, hav_out, hav_in, s0, l0, s1, l1);
            else
                band_window(bd, a.cell_start, f.th, f.sh, f.ch, f.inv_sp, f.phf, hav_out, hav_in, s0, l0, s1, l1);
            const int base = 2 * bd.pt_start;
#pragma unroll
            for (int seg = 0; seg < 2; ++seg) {
                int j = base + (seg == 0 ? s0 : s1);
                const int jend = j + (seg == 0 ? l0 : l1);
                // the wave's span of this segment; inactive lanes do not widen it
                const bool any = j < jend;
                const int jlo = __builtin_amdgcn_readfirstlane(wave_min(any ? j : 0x7fffffff));
                const int jhi = __builtin_amdgcn_readfirstlane(wave_max(any ? jend : -1));
                if (jhi <= jlo) continue;
                const bool use_lds = jhi - jlo <= SLOTS;
                for (; j < jend; ++j) {
                    const double4 r = a.rec[j];
                    const double dx = r.x - f.xp, dy = r.y - f.yp, dz = r.z - f.zp;
                    const double d2 = (dx * dx + dy * dy) + dz * dz;
                    if (d2 >= elo && d2 < ehi) {
                        const double u1 = fma(dx, f.nx, fma(dy, f.ny, dz * f.nz));
                        const double u2 = fma(dx, f.ex, dy * f.ey);
                        double tc, ts;  // 2 cos(phi), 2 sin(phi)
                        twice_unit_bearing(u1, u2, kBearingTiny, tc, ts);
                        // sum_m Re(exp(-i m phi) D(m)) = sum_m cos(m phi) Re D + sin(m phi) Im D
                        double acc[K];
#pragma unroll
                        for (int k = 0; k < K; ++k) acc[k] = M >= 1 ? fma(ts, Bt[k][0], Al[k][0]) : Al[k][0];
                        if constexpr (M >= 1) {
                            double ua = 1.0, ub = tc;  // U_0, U_1
#pragma unroll
                            for (int m = 1; m <= M; ++m) {
#pragma unroll
                                for (int k = 0; k < K; ++k)
                                    acc[k] = fma(ub, m < M ? fma(ts, Bt[k][m], Al[k][m]) : Al[k][m], acc[k]);
                                if (m < M) {
                                    const double um = fma(tc, ub, -ua);
                                    ua = ub; ub = um;
                                }
                            }
                        }
                        if (!unit_w) {
                            const double wj = a.wdbl[j];
#pragma unroll
                            for (int k = 0; k < K; ++k) acc[k] *= wj;
                        }
                        if (use_lds) {
#pragma unroll
                            for (int k = 0; k < K; ++k) atomicAdd(&agg[k][j - jlo], acc[k]);
                        } else {
                            int t = j - base;
                            if (t >= bd.npts) t -= bd.npts;
#pragma unroll
                            for (int k = 0; k < K; ++k)
                                atomicAdd(&a.grad[(mp0 + k) * a.n_stride + bd.pt_start + t], acc[k]);
                        }
                    }
                }
                if (use_lds) {
                    // one global atomic per touched neighbour and map, and the slice is cleared
                    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS adds are done
                    __builtin_amdgcn_wave_barrier();
                    for (int e = lane; e < jhi - jlo; e += kWave) {
                        int t = jlo + e - base;
                        if (t >= bd.npts) t -= bd.npts;
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            const double val = agg[k][e];
                            if (val != 0.0) {
                                atomicAdd(&a.grad[(mp0 + k) * a.n_stride + bd.pt_start + t], val);
                                agg[k][e] = 0.0;
                            }
                        }
                    }
                    __builtin_amdgcn_s_waitcnt(0xc07f);
                    __builtin_amdgcn_wave_barrier();
                }
            }
        }
    }
}

__global__ void k_grad_to_catalogue(int64_t n, const int *perm, const double *gs, double *grad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) grad[perm[i]] += gs[i];
}

// Maps in pairs (geometry shared by two maps per lane), an odd last map alone.
template <int M>
static void launch_scatter_m(const ScatterArgs &a, int nm, bool planar, hipStream_t s)
{
    if (planar) {  // one map per lane, one grid row per map
        hipLaunchKernelGGL((k_adjoint_scatter<M, 1, true>), dim3(a.nblocks, nm), dim3(kBlock), 0, s, a);
        return;
    }
    if (nm >= 4) hipLaunchKernelGGL((k_adjoint_scatter<M, 4>), dim3(a.nblocks, nm / 4), dim3(kBlock), 0, s, a);
    if (nm & 2) {
        ScatterArgs b = a;
        const size_t first = (size_t)(nm & ~3);
        b.pv += first * a.n_stride;
        b.grad += first * a.n_stride;
        b.rec += first * a.rec_stride;
        b.D += first * a.d_stride;
        hipLaunchKernelGGL((k_adjoint_scatter<M, 2>), dim3(a.nblocks, 1), dim3(kBlock), 0, s, b);
    }
    if (nm & 1) {
        ScatterArgs b = a;
        const size_t last = (size_t)(nm - 1);
        b.pv += last * a.n_stride;
        b.grad += last * a.n_stride;
        b.rec += last * a.rec_stride;
        b.D += last * a.d_stride;
        hipLaunchKernelGGL((k_adjoint_scatter<M, 1>), dim3(a.nblocks, 1), dim3(kBlock), 0, s, b);
    }
}

// Prep + scatter of maps [map, map + nm) for pivots [c0, c1) whose multipoles A (ld =
// c1 - c0, maps `stride` elements apart) and weights W are already in the workspace; D has
// the layout of A.  G and gs (index-order gradients, idx->n apart) start at map `map`.
static z3_status adjoint_chunk_maps(z3_index idx, int map, int nm, int m_max, int64_t c0, int64_t c1,
                                    const double *A, size_t stride, const double *W, const double *G, double scale,
                                    double *D, double *gs, hipStream_t s)
{
    const int64_t P = c1 - c0;
    const double *vmap = idx->d_v + (size_t)map * idx->n;
    const size_t gstride = (size_t)(m_max + 1) * idx->nbins * idx->nbins * 2;
    PrepArgs pa;
    pa.A = A;
    pa.W = W;
    pa.G = G;
    pa.v = vmap + c0;
    pa.w = idx->d_w + c0;
    pa.D = D;
    pa.grad = gs + c0;
    pa.P = P;
    pa.nb = idx->nbins;
    pa.M = m_max;
    pa.scale = scale;
    pa.ad_stride = stride;
    pa.g_stride = gstride;
    pa.n_stride = (size_t)idx->n;
    const dim3 pgrid((unsigned)((P + 255) / 256), nm);
    if (idx->nbins <= 16) hipLaunchKernelGGL(k_adjoint_prep<16>, pgrid, dim3(256), 0, s, pa);
    else if (idx->nbins <= 32) hipLaunchKernelGGL(k_adjoint_prep<32>, pgrid, dim3(256), 0, s, pa);
    else hipLaunchKernelGGL(k_adjoint_prep_any, pgrid, dim3(256), 0, s, pa);
    z3_status st = check_launch("k_adjoint_prep");
    if (st != Z3_OK) return st;
    ScatterArgs sa;
    sa.px = idx->d_x; sa.py = idx->d_y; sa.pz = idx->d_z;
    sa.pv = vmap;
    sa.rec = idx->d_rec + (size_t)map * 2 * idx->n;
    sa.wdbl = idx->unit_w ? nullptr : idx->d_wdbl;
    sa.cell_start = idx->d_cell_start;
    sa.bands = idx->d_bands;
    sa.nbands = idx->nbands;
    sa.inv_h = 1.0 / idx->band_h;
    sa.edges = idx->d_edges;
    sa.nb = idx->nbins;
    sa.p0 = c0; sa.p1 = c1;
    sa.D = D;
    sa.ldD = P;
    sa.grad = gs;
    sa.scale = scale;
    sa.nblocks = (int)((P + kBlock - 1) / kBlock);
    sa.n_stride = (size_t)idx->n;
    sa.rec_stride = (size_t)2 * idx->n;
    sa.d_stride = stride;
    sa.px0 = idx->plane_x0; sa.py0 = idx->plane_y0; sa.psx = idx->plane_sx;
    switch (m_max) {
#define Z3_CASE(MM) case MM: launch_scatter_m<MM>(sa, nm, idx->planar, s); break;
        Z3_CASE(0) Z3_CASE(1) Z3_CASE(2) Z3_CASE(3) Z3_CASE(4) Z3_CASE(5) Z3_CASE(6) Z3_CASE(7)
        Z3_CASE(8) Z3_CASE(9) Z3_CASE(10) Z3_CASE(11) Z3_CASE(12) Z3_CASE(13) Z3_CASE(14)
        Z3_CASE(15) Z3_CASE(16)
#undef Z3_CASE
    default: st = fail(Z3_ERR_UNSUPPORTED, "m_max=%d not compiled", m_max);
    }
    if (st == Z3_OK) st = check_launch("k_adjoint_scatter");
    return st;
}

static z3_status grad_to_catalogue(z3_index idx, const double *gs, double *grad_x, hipStream_t s)
{
    if (idx->n == 0) return Z3_OK;
    hipLaunchKernelGGL(k_grad_to_catalogue, dim3((unsigned)((idx->n + 255) / 256)), dim3(256), 0, s, idx->n,
                       idx->d_perm, gs, grad_x);
    return check_launch("k_grad_to_catalogue");
}

z3_status adjoint_impl(z3_index idx, int map, int m_max, int64_t p0, int64_t p1, const double *G, double scale,
                       double *grad_x, hipStream_t s, int64_t chunk)
{
    ProfileMute mute;  // the recomputed multipoles are not forward launches
    const int nb = idx->nbins;
    if (chunk > p1 - p0) chunk = ((p1 - p0 + kBlock - 1) / kBlock) * kBlock;
    if (chunk < kBlock) chunk = kBlock;
    const size_t per_piv = (size_t)(m_max + 1) * 2 * nb;
    void *wa = nullptr, *wd = nullptr, *ww = nullptr, *wg = nullptr;
    z3_status st = scratch_alloc(&wa, (size_t)chunk * per_piv * sizeof(double), s);
    if (st == Z3_OK) st = scratch_alloc(&wd, (size_t)chunk * per_piv * sizeof(double), s);
    if (st == Z3_OK) st = scratch_alloc(&ww, (size_t)chunk * nb * sizeof(double), s);
    if (st == Z3_OK) st = scratch_alloc(&wg, (size_t)idx->n * sizeof(double), s);
    if (st == Z3_OK) st = launch_fill(static_cast<double *>(wg), idx->n, 0.0, s);
    double *gs = static_cast<double *>(wg);
    for (int64_t c0 = p0; c0 < p1 && st == Z3_OK; c0 += chunk) {
        const int64_t c1 = c0 + chunk < p1 ? c0 + chunk : p1;
        st = launch_multipoles(idx, Pivots{idx->d_x, idx->d_y, idx->d_z}, map, m_max, Z3_PREC_FP64, Z3_NORM_BIN, c0,
                               c1, wa, c1 - c0, static_cast<double *>(ww), nullptr, nullptr, nullptr, s);
        if (st == Z3_OK)
            st = adjoint_chunk_maps(idx, map, 1, m_max, c0, c1, static_cast<const double *>(wa), 0,
                                    static_cast<const double *>(ww), G, scale, static_cast<double *>(wd), gs, s);
    }
    if (st == Z3_OK) st = grad_to_catalogue(idx, gs, grad_x, s);
    scratch_free(wg, s);
    scratch_free(ww, s);
    scratch_free(wd, s);
    scratch_free(wa, s);
    return st;
}

// All attached maps.  Their multipoles are recomputed group by group (kMapGroup maps) by the
// register-tiled many-map kernel, or, for many maps (many_maps_on_mfma), by the MFMA
// many-map kernel, all maps of a pivot chunk at once.  Then one prep and one scatter launch
// cover every map of the pass.
// `budget` is the pivot count whose single-map FP64 multipoles fill the workspace budget.
z3_status adjoint_maps_impl(z3_index idx, int m_max, int64_t p0, int64_t p1, const double *G, double scale,
                            double *grad_x, hipStream_t s, int64_t budget)
{
    ProfileMute mute;  // the recomputed multipoles are not forward launches
    const int nb = idx->nbins;
    const bool batch = many_maps_on_mfma(idx, Z3_PREC_FP64);  // the recompute runs in FP64
    int shape = 0;
    z3_status st = Z3_OK;
    if (batch && (st = batch_shape(idx, m_max, Z3_PREC_FP64, p0, p1, s, &shape)) != Z3_OK) return st;
    const int per_pass = batch ? idx->nmaps : kMapGroup;  // multipole sets held at once
    int64_t chunk = budget / (2 * per_pass);               // A and D of every map of the pass
    chunk = (chunk / kBlock) * kBlock;
    if (chunk < kBlock) chunk = kBlock;
    if (chunk > p1 - p0) chunk = ((p1 - p0 + kBlock - 1) / kBlock) * kBlock;
    const size_t per_piv = (size_t)(m_max + 1) * 2 * nb;
    const size_t gstride = (size_t)(m_max + 1) * nb * nb * 2;
    void *wa = nullptr, *wd = nullptr, *ww = nullptr, *wg = nullptr;
    st = scratch_alloc(&wa, (size_t)per_pass * chunk * per_piv * sizeof(double), s);
    if (st == Z3_OK) st = scratch_alloc(&wd, (size_t)per_pass * chunk * per_piv * sizeof(double), s);
    if (st == Z3_OK) st = scratch_alloc(&ww, (size_t)chunk * nb * sizeof(double), s);
    if (st == Z3_OK) st = scratch_alloc(&wg, (size_t)idx->nmaps * idx->n * sizeof(double), s);
    if (st == Z3_OK) st = launch_fill(static_cast<double *>(wg), (int64_t)idx->nmaps * idx->n, 0.0, s);
    // one or two maps left over after the full groups run one-map adjoints (cheaper than a
    // group pass), once the groups' workspace is released
    const int rest = batch ? 0 : (idx->nmaps % kMapGroup <= 2 ? idx->nmaps % kMapGroup : 0);
    const int ngroups = batch ? 1 : (idx->nmaps - rest + kMapGroup - 1) / kMapGroup;
    for (int g = 0; g < ngroups && st == Z3_OK; ++g) {
        const int map0 = g * kMapGroup;
        const int nm = batch ? idx->nmaps : (idx->nmaps - map0 < kMapGroup ? idx->nmaps - map0 : kMapGroup);
        for (int64_t c0 = p0; c0 < p1 && st == Z3_OK; c0 += chunk) {
            const int64_t c1 = c0 + chunk < p1 ? c0 + chunk : p1;
            const size_t stride = (size_t)(c1 - c0) * per_piv;
            if (batch)
                // wd (written later by the prep) stages the pivot-major multipoles
                st = launch_multipoles_batch(idx, m_max, Z3_PREC_FP64, shape, c0, c1, wd, wa, c1 - c0, stride,
                                             static_cast<double *>(ww), nullptr, s);
            else
                st = launch_multipoles_maps(idx, g, nm, m_max, Z3_PREC_FP64, c0, c1, wa, c1 - c0, stride,
                                            static_cast<double *>(ww), nullptr, s);
            if (st == Z3_OK)
                st = adjoint_chunk_maps(idx, map0, nm, m_max, c0, c1, static_cast<const double *>(wa), stride,
                                        static_cast<const double *>(ww), G + map0 * gstride, scale,
                                        static_cast<double *>(wd), static_cast<double *>(wg) + (size_t)map0 * idx->n,
                                        s);
        }
    }
    for (int map = 0; map < idx->nmaps - rest && st == Z3_OK; ++map)
        st = grad_to_catalogue(idx, static_cast<double *>(wg) + (size_t)map * idx->n, grad_x + (size_t)map * idx->n, s);
    scratch_free(wg, s);
    scratch_free(ww, s);
    scratch_free(wd, s);
    scratch_free(wa, s);
    for (int k = idx->nmaps - rest; k < idx->nmaps && st == Z3_OK; ++k)
        st = ::z3_adjoint(idx, k, m_max, p0, p1, G + k * gstride, scale, grad_x + (size_t)k * idx->n, s);
    return st;
}

}  // namespace z3
