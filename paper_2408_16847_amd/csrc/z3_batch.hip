// Many-map multipoles on MFMA (eqs. Xm.binned, Ym/Zm for a batch of fields that share
// positions and weights).
//
// For one pivot p and bin b, every map mu needs
//     a_{m,b}(p; mu) = sum_j v_j(mu) e^{-i m phi_pj},      v_j(mu) = w_j x_j(mu),
// which, over the candidates j of the pivot's windows, is the product
//     C[mu][c] = sum_j V[j][mu] H[j][c],   H[j] = [1, cos phi, .., cos M phi, sin phi, .., sin M phi]
// masked to the pairs that fall in bin b.  The geometry (distance, bin, bearing, the
// Chebyshev harmonics) is computed once per pair and shared by all maps; the sum over
// pairs is a dense [maps x pairs] x [pairs x (2M+1)] contraction and runs on MFMA.
//
// Work split: one block owns one pivot and 16 * TI * WPB maps (WPB wave64s, 16 * TI maps
// per wave).  The windows of up to 64 bands are laid end to end (one band per lane of
// the first wave, prefix sum of the window lengths).  Groups of 64 * WPB consecutive
// candidates then go one per thread: each thread tests its candidate and writes its
// harmonic row to LDS; after a block barrier every wave runs the MFMA steps for its own
// maps over the whole group, 4 candidates per step: A = map values (16 maps x 4
// candidates, read from the per-record value matrix), B = harmonic rows (4 candidates x
// 16 columns, from LDS).  The shape (WPB, TI) is a tuning choice.
//
// Precision: FP64 path: FP64 harmonics, values and v_mfma_f64_16x16x4f64 accumulation.
// Mixed path: harmonics computed in FP64 and rounded to FP32, FP32 values, and
// v_mfma_f32_16x16x4f32; the FP32 sums over each run of 128 candidates are added into
// FP64 bin sums.  Distances and bin decisions are FP64 on both paths (bit-exact pair sets).
#include "z3_batch_device.h"

namespace z3 {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

struct BatchArgs {
    const double4 *rec;           // [2n] doubled records (x, y, z, .)
    const void *vmat;             // [2n][ldv] doubled per-map values w * x (FP64 or FP32)
    int ldv;                      // maps padded to a multiple of 32 (zeros)
    const double *wdbl;           // [2n] doubled weights, or null for unit weights
    const int *cell_start;
    const Band *bands;
    int nbands;
    double inv_h;
    const EdgeTab *edges;
    int nb;
    const double *px, *py, *pz;   // pivots (index order)
    int64_t p0, p1;
    int nmaps;                    // maps written (rows >= nmaps are padding)
    int ntiles;                   // map tiles of one pivot (blocks per pivot)
    void *stage;                  // [P][nb][nmaps][2 (m+1)] pivot-major multipoles (re, im per m)
    double *W;                    // [nb][ldA] W_{p,b}, or null
    int64_t ldA;
    uint64_t *pair_total;
    int nblocks;
};

// Block shapes the library is built with: waves per block, 16-map tiles per wave.
struct BatchShape { int wpb, ti; };
constexpr BatchShape kBatchShapes[] = {{4, 1}, {2, 2}, {2, 1}, {4, 2}};
constexpr int kNumBatchShapes = sizeof(kBatchShapes) / sizeof(kBatchShapes[0]);

template <bool F32> struct BatchT { typedef double T; typedef v4d V4; };
template <> struct BatchT<true> { typedef float T; typedef v4f V4; };

// Register budget: 3 waves per SIMD on the mixed path (measured faster than the
// compiler's own choice), 2 on the FP64 path.
template <int M, bool F32, int WPB, int TI>
__global__ __launch_bounds__(WPB * kWave) __attribute__((amdgpu_waves_per_eu(F32 ? 3 : 2)))
void k_multipoles_batch(BatchArgs a)
{
    typedef typename BatchT<F32>::T T;
    typedef typename BatchT<F32>::V4 V4;
    constexpr int NC = 2 * M + 1;             // harmonic columns
    constexpr int NCT = (NC + 15) / 16;       // 16-column MFMA tiles
    constexpr int HS = (NC + 31) / 32 * 32;   // LDS row length of the harmonic rows
    constexpr int NCAND = WPB * kWave;        // candidates per group

    __shared__ int s_bend[kWave], s_a0[kWave], s_a1[kWave], s_split[kWave];
    __shared__ int s_total;
    __shared__ int s_j[NCAND];
    __shared__ T s_h[NCAND * HS];
    __shared__ int s_cnt[WPB];
    __shared__ double s_wc[NCAND];  // weights of the group's candidates (0 outside the bin)
    __shared__ double s_W;

    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int tid = threadIdx.x;
    // logical block: XCD-contiguous; the map tiles of one pivot are adjacent
    const int lb = xcd_block(blockIdx.x, a.nblocks);
    const int mt = lb % a.ntiles;
    const int64_t p = a.p0 + lb / a.ntiles;
    if (p >= a.p1) return;  // uniform per block
    const int mb = (mt * WPB + wv) * 16 * TI;  // first map of this wave
    const bool has_maps = mb < a.nmaps;        // uniform per wave

    const PivotFrame f = uniform_frame(pivot_frame(a.px[p], a.py[p], a.pz[p]));
    const int64_t col = p - a.p0;
    const int nb = a.nb;
    const bool unit_w = a.wdbl == nullptr;
    const int r16 = lane & 15, g4 = lane >> 4;
    const T *vm = static_cast<const T *>(a.vmat) + (has_maps ? mb + TI * r16 : 0);
    uint64_t pairs_all = 0;

    for (int bin = 0; bin < nb; ++bin) {
        const double elo = a.edges->e[bin], ehi = a.edges->e[bin + 1];
        const double hav_out = a.edges->hav_out[bin + 1], hav_in = a.edges->hav_in[bin];
        const double rad = a.edges->rad_out[bin + 1];
        const int klo = max((int)floor((f.th - rad) * a.inv_h), 0);
        const int khi = min((int)floor((f.th + rad) * a.inv_h), a.nbands - 1);

        V4 acc[TI][NCT];
        double acc64[TI][NCT][4];
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int t = 0; t < NCT; ++t) {
                acc[i][t] = V4{0, 0, 0, 0};
#pragma unroll
                for (int r = 0; r < 4; ++r) acc64[i][t][r] = 0.0;
            }
        double wslot = 0.0;  // first wave: weight sum of candidates lane, lane + 64, ...
        int cnt = 0;

        for (int kb = klo; kb <= khi; kb += kWave) {
            if (wv == 0) {
                // one band per lane: its window segments, laid end to end
                const int k = kb + lane;
                int s0 = 0, l0 = 0, s1 = 0, l1 = 0, base = 0;
                if (k <= khi) {
                    const Band bd = a.bands[k];
                    if (bd.npts > 0) {
                        band_window(bd, a.cell_start, f.th, f.sh, f.ch, f.inv_sp, f.phf, hav_out, hav_in, s0, l0,
                                    s1, l1);
                        base = 2 * bd.pt_start;
                    }
                }
                const int len = l0 + l1;
                const int incl = wave_incl_scan(len, lane);
                const int excl = incl - len;
                s_bend[lane] = incl;
                s_a0[lane] = base + s0 - excl;
                s_split[lane] = excl + l0;
                s_a1[lane] = base + s1 - (excl + l0);
                if (lane == kWave - 1) s_total = incl;
            }
            __syncthreads();
            const int total = s_total;

            for (int f0 = 0; f0 < total; f0 += NCAND) {
                // locate this thread's candidate: band slot = first q with s_bend[q] > fc
                // (s_bend is non-decreasing and s_bend[63] = total)
                const int fi = f0 + tid;
                const bool cand = fi < total;
                const int fc = cand ? fi : total - 1;
                int q = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1)
                    if (s_bend[q + step - 1] <= fc) q += step;
                const int j = fc < s_split[q] ? s_a0[q] + fc : s_a1[q] + fc;

                const double4 rec = a.rec[j];
                const double dx = rec.x - f.xp, dy = rec.y - f.yp, dz = rec.z - f.zp;
                const double d2 = (dx * dx + dy * dy) + dz * dz;
                const bool in = cand && d2 >= elo && d2 < ehi;
                T h[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) h[c] = T(0);
                if (!unit_w) s_wc[tid] = in ? a.wdbl[j] : 0.0;
                if (in) {
                    cnt += 1;
                    const double u1 = fma(dx, f.nx, fma(dy, f.ny, dz * f.nz));
                    const double u2 = fma(dx, f.ex, dy * f.ey);
                    double c1, sn1;
                    unit_bearing(u1, u2, c1, sn1);
                    // cos(m phi) = T_m(cos phi), sin(m phi) = sin phi U_{m-1}(cos phi): the
                    // three-term recurrence in FP64 on both paths (as cheap as FP32 on this
                    // hardware, and free of the recurrence's error growth in FP32); the mixed
                    // path rounds each harmonic to FP32 once
                    h[0] = T(1);
                    if constexpr (M >= 1) {
                        const double tc = c1 + c1;
                        double t2 = 1.0, t1 = c1, u2s = 0.0, u1s = sn1;
                        h[1] = (T)t1;
                        h[M + 1] = (T)u1s;
#pragma unroll
                        for (int m = 2; m <= M; ++m) {
                            const double tm = fma(tc, t1, -t2);
                            const double sm = fma(tc, u1s, -u2s);
                            h[m] = (T)tm;
                            h[M + m] = (T)sm;
                            t2 = t1; t1 = tm;
                            u2s = u1s; u1s = sm;
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) s_h[hslot<HS>(tid, c)] = h[c];
                s_j[tid] = j;
                __syncthreads();
                if (!unit_w && wv == 0) {
                    // W_{p,b} summed per candidate slot in candidate order, the same for
                    // every block shape
#pragma unroll
                    for (int w = 0; w < WPB; ++w) wslot += s_wc[w * kWave + lane];
                }

                if (has_maps) {
                    // MFMA steps of 4 candidates over the group's filled part.  The map values
                    // are fetched PF steps ahead (their addresses come from the LDS index list,
                    // their latency is that of L2/HBM).  The mixed path adds its FP32 sums into
                    // the FP64 bin sums every 32 steps (128 candidates of the band batch), the
                    // same points for every block shape.
                    constexpr int PF = TI == 1 ? 16 : 8;
                    const int nst = (min(total - f0, NCAND) + 3) >> 2;
                    T vbuf[PF][TI];
#pragma unroll
                    for (int d = 0; d < PF; ++d) {
                        if (d < nst) {
                            const T *vp = vm + (size_t)s_j[4 * d + g4] * a.ldv;
#pragma unroll
                            for (int i = 0; i < TI; ++i) vbuf[d][i] = vp[i];
                        }
                    }
                    for (int st0 = 0; st0 < nst; st0 += PF) {
#pragma unroll
                        for (int u = 0; u < PF; ++u) {
                            const int st = st0 + u;
                            if (st < nst) {
                                const int src = 4 * st + g4;
                                T hb[NCT];
#pragma unroll
                                for (int t = 0; t < NCT; ++t) {
                                    const int c = 16 * t + r16;
                                    hb[t] = c < NC ? s_h[hslot<HS>(src, c)] : T(0);
                                }
#pragma unroll
                                for (int i = 0; i < TI; ++i)
#pragma unroll
                                    for (int t = 0; t < NCT; ++t) {
                                        if constexpr (F32)
                                            acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(vbuf[u][i], hb[t], acc[i][t],
                                                                                             0, 0, 0);
                                        else
                                            acc[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(vbuf[u][i], hb[t], acc[i][t],
                                                                                             0, 0, 0);
                                    }
                                if (st + PF < nst) {
                                    const T *vp = vm + (size_t)s_j[4 * (st + PF) + g4] * a.ldv;
#pragma unroll
                                    for (int i = 0; i < TI; ++i) vbuf[u][i] = vp[i];
                                }
                                if constexpr (F32) {
                                    if ((st & 31) == 31 || st == nst - 1) {
#pragma unroll
                                        for (int i = 0; i < TI; ++i)
#pragma unroll
                                            for (int t = 0; t < NCT; ++t) {
#pragma unroll
                                                for (int r = 0; r < 4; ++r) acc64[i][t][r] += (double)acc[i][t][r];
                                                acc[i][t] = V4{0, 0, 0, 0};
                                            }
                                    }
                                }
                            }
                        }
                    }
                }
                __syncthreads();  // the next group overwrites the rows and indices
            }
            __syncthreads();  // the band table and s_total are rewritten next
        }

        // the pair count over the block; W_{p,b} from the first wave's slot sums
        {
            const int cw = wave_sum_i32(cnt);
            if (lane == 0) s_cnt[wv] = cw;
            if (!unit_w && wv == 0) {
                const double wt = wave_sum_f64(wslot);
                if (lane == 0) s_W = wt;
            }
        }
        __syncthreads();
        int cnt_b = 0;
#pragma unroll
        for (int w = 0; w < WPB; ++w) cnt_b += s_cnt[w];
        const double Wb = unit_w ? (double)cnt_b : s_W;
        pairs_all += (uint64_t)cnt_b;
        if (has_maps) {
            const double inv = Wb > 0.0 ? 1.0 / Wb : 0.0;
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int t = 0; t < NCT; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        // f32 16x16x4 result: register r of lane l is D[4 (l/16) + r][l % 16];
                        // f64 16x16x4 result: register r of lane l is D[4 r + l/16][l % 16]
                        const int row = F32 ? 4 * g4 + r : 4 * r + g4;
                        const int c = 16 * t + r16;
                        const int map = mb + TI * row + i;
                        if (map >= a.nmaps || c > NC) continue;
                        const double s = F32 ? acc64[i][t][r] : (double)acc[i][t][r];
                        int m, part;
                        double val;
                        if (c == NC) { m = 0; part = 1; val = 0.0; }            // Im X_0 = 0
                        else if (c == 0) { m = 0; part = 0; val = s * inv; }
                        else if (c <= M) { m = c; part = 0; val = s * inv; }
                        else { m = c - M; part = 1; val = -s * inv; }        // e^{-i m phi}
                        // pivot-major staging: the bin's values of all maps are one contiguous
                        // run, so the block's stores fill whole cache lines
                        const size_t o = (((size_t)col * nb + bin) * (size_t)a.nmaps + map) * (2 * (M + 1)) + 2 * m + part;
                        static_cast<T *>(a.stage)[o] = (T)val;
                    }
        }
        if (mt == 0 && tid == 0 && a.W) a.W[(size_t)bin * (size_t)a.ldA + col] = Wb;
    }
    if (mt == 0 && tid == 0 && a.pair_total && pairs_all)
        atomicAdd((unsigned long long *)a.pair_total, (unsigned long long)pairs_all);
}

template <int M, bool F32, int S>
static void launch_shape(const BatchArgs &a, hipStream_t s)
{
    constexpr int WPB = kBatchShapes[S].wpb, TI = kBatchShapes[S].ti;
    hipLaunchKernelGGL((k_multipoles_batch<M, F32, WPB, TI>), dim3(a.nblocks), dim3(WPB * kWave), 0, s, a);
}

template <int M, bool F32>
static z3_status launch_batch_m(int shape, const BatchArgs &a, hipStream_t s)
{
    switch (shape) {
    case 0: launch_shape<M, F32, 0>(a, s); break;
    case 1: launch_shape<M, F32, 1>(a, s); break;
    case 2: launch_shape<M, F32, 2>(a, s); break;
    case 3: launch_shape<M, F32, 3>(a, s); break;
    default: return fail(Z3_ERR_UNSUPPORTED, "batch shape %d not compiled", shape);
    }
    return Z3_OK;
}

int batch_ldv(int nmaps) { return (nmaps + 31) / 32 * 32; }  // whole 32-map wave tiles
int batch_num_shapes() { return kNumBatchShapes; }
void batch_shape_dims(int shape, int *wpb, int *ti)
{
    *wpb = kBatchShapes[shape].wpb;
    *ti = kBatchShapes[shape].ti;
}

// Pivot-major staging [P][nb][nmaps][R] -> A [map][R][nb][ldA] (R = 2 (m+1) rows re/im per
// m; row r of bin b is row r nb + b): one block per (64 pivots, bin, map), through LDS, so
// both the reads (runs of R values per pivot) and the writes (runs of 64 pivots) are
// contiguous.
constexpr int kMaxRows = 2 * (Z3_MAX_MMAX + 1);

template <class T>
__global__ __launch_bounds__(256) void k_batch_transpose(const T *stage, T *A, int64_t P, int nb, int nmaps, int R,
                                                         int64_t ldA, size_t map_stride)
{
    __shared__ T tile[kMaxRows][65];
    const int64_t pt0 = (int64_t)blockIdx.x * 64;
    const int b = blockIdx.y, map = blockIdx.z;
    const int np = (int)(P - pt0 < 64 ? P - pt0 : 64);
    for (int e = threadIdx.x; e < np * R; e += 256) {
        const int pl = e / R, r = e - pl * R;
        tile[r][pl] = stage[(((size_t)(pt0 + pl) * nb + b) * nmaps + map) * R + r];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < R * 64; e += 256) {
        const int r = e / 64, pl = e - r * 64;
        if (pl < np) A[(size_t)map * map_stride + ((size_t)r * nb + b) * ldA + pt0 + pl] = tile[r][pl];
    }
}

z3_status launch_multipoles_batch(const z3_index_s *idx, int m_max, int prec, int shape, int64_t p0, int64_t p1,
                                  void *stage, void *A, int64_t ldA, size_t map_stride, double *W,
                                  uint64_t *pair_total, hipStream_t s)
{
    if (shape < 0 || shape >= kNumBatchShapes) return fail(Z3_ERR_INVALID_ARG, "batch shape %d", shape);
    const int per_block = 16 * kBatchShapes[shape].ti * kBatchShapes[shape].wpb;
    const int ntiles = (batch_ldv(idx->nmaps) + per_block - 1) / per_block;
    const int R = 2 * (m_max + 1);
    const bool f32 = prec == Z3_PREC_MIXED;
    if (p1 <= p0) return Z3_OK;
    if (idx->nmaps > 65535) return fail(Z3_ERR_UNSUPPORTED, "more than 65535 maps");
    // one launch stays well below 2^32 work-items: at most 2^22 blocks
    const int64_t max_piv = ((int64_t)1 << 22) / ntiles;
    if (p1 - p0 > max_piv) {
        for (int64_t c0 = p0; c0 < p1; c0 += max_piv) {
            const int64_t c1 = c0 + max_piv < p1 ? c0 + max_piv : p1;
            const size_t off = (size_t)(c0 - p0);
            const size_t soff = off * idx->nbins * idx->nmaps * R;
            z3_status st;
            if (f32)
                st = launch_multipoles_batch(idx, m_max, prec, shape, c0, c1, static_cast<float *>(stage) + soff,
                                             A ? static_cast<float *>(A) + off : nullptr, ldA, map_stride,
                                             W ? W + off : nullptr, pair_total, s);
            else
                st = launch_multipoles_batch(idx, m_max, prec, shape, c0, c1, static_cast<double *>(stage) + soff,
                                             A ? static_cast<double *>(A) + off : nullptr, ldA, map_stride,
                                             W ? W + off : nullptr, pair_total, s);
            if (st != Z3_OK) return st;
        }
        return Z3_OK;
    }
    const int64_t nblk = (p1 - p0) * ntiles;
    BatchArgs a;
    a.rec = idx->d_rec;
    a.vmat = f32 ? static_cast<const void *>(idx->d_vmat32) : static_cast<const void *>(idx->d_vmat64);
    a.ldv = batch_ldv(idx->nmaps);
    a.wdbl = idx->unit_w ? nullptr : idx->d_wdbl;
    a.cell_start = idx->d_cell_start;
    a.bands = idx->d_bands;
    a.nbands = idx->nbands;
    a.inv_h = 1.0 / idx->band_h;
    a.edges = idx->d_edges;
    a.nb = idx->nbins;
    a.px = idx->d_x; a.py = idx->d_y; a.pz = idx->d_z;
    a.p0 = p0; a.p1 = p1;
    a.nmaps = idx->nmaps;
    a.ntiles = ntiles;
    a.stage = stage;
    a.W = W;
    a.ldA = ldA;
    a.pair_total = pair_total;
    a.nblocks = (int)nblk;
    hipEvent_t ev0;
    profile_begin(s, &ev0);
    z3_status st = Z3_OK;
    switch (m_max) {
#define Z3_CASE(MM) \
    case MM: st = f32 ? launch_batch_m<MM, true>(shape, a, s) : launch_batch_m<MM, false>(shape, a, s); break;
        Z3_CASE(0) Z3_CASE(1) Z3_CASE(2) Z3_CASE(3) Z3_CASE(4) Z3_CASE(5) Z3_CASE(6) Z3_CASE(7)
        Z3_CASE(8) Z3_CASE(9) Z3_CASE(10) Z3_CASE(11) Z3_CASE(12) Z3_CASE(13) Z3_CASE(14)
        Z3_CASE(15) Z3_CASE(16)
#undef Z3_CASE
    default: st = fail(Z3_ERR_UNSUPPORTED, "m_max=%d not compiled", m_max);
    }
    if (st == Z3_OK) st = check_launch("k_multipoles_batch");
    profile_end(s, ev0);
    if (st != Z3_OK || !A) return st;
    const dim3 tgrid((unsigned)((p1 - p0 + 63) / 64), (unsigned)idx->nbins, (unsigned)idx->nmaps);
    if (f32)
        hipLaunchKernelGGL(k_batch_transpose<float>, tgrid, dim3(256), 0, s, static_cast<const float *>(stage),
                           static_cast<float *>(A), p1 - p0, idx->nbins, idx->nmaps, R, ldA, map_stride);
    else
        hipLaunchKernelGGL(k_batch_transpose<double>, tgrid, dim3(256), 0, s, static_cast<const double *>(stage),
                           static_cast<double *>(A), p1 - p0, idx->nbins, idx->nmaps, R, ldA, map_stride);
    return check_launch("k_batch_transpose");
}

}  // namespace z3
