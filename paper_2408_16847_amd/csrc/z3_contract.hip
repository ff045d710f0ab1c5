// Contraction of the per-pivot multipoles (eqs. zetamEst, zetamEst2) on MFMA.
//
// For every m, with U_p = [Re X_m(0..nb-1; p), Im X_m(0..nb-1; p)] (length 2 nb):
//     G = sum_p v_p U_p U_p^T                       (2nb x 2nb real Gram matrix)
//     Re zeta_m(b1, b2) = G(r1, r2) + G(i1, i2),   Im zeta_m(b1, b2) = G(i1, r2) - G(r1, i2)
// (r = b, i = nb + b), which is sum_p v_p X(b1) conj(X(b2)) written in real arithmetic.
// The Gram matrix is a dense contraction over pivots, formed in 16 x 16 tiles over segments
// of pivots with v_mfma_f64_16x16x4f64 (FP64 path) or v_mfma_f32_16x16x4f32 (mixed path: FP32
// multipoles U; the scaled operand v_p U_i is formed in FP64 and split into FP32 hi + lo
// parts, two MFMAs per step; FP32 sums over 16 pivots are added into FP64 segment sums),
// from tiles of pivots staged in LDS (k_pair_lds for the pivot-minor layout of the one-map
// kernels, k_gram_lds for the many-map kernel's pivot-major staging).
// Only tiles on or above the diagonal are formed; entries below are read from their
// mirror, so zeta(b2, b1) is exactly conj(zeta(b1, b2)) and Im zeta(b, b) is exactly 0.
// Segment partials are summed in FP64 in segment order (deterministic).
#include <algorithm>
#include <type_traits>

#include "z3_internal.h"

namespace z3 {

constexpr int kSeg = 4096;  // pivots per contraction wave

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

static inline int tiles_for(int nbins) { return (2 * nbins + 15) / 16; }

size_t contract_partial_bytes(int64_t npiv, int m_max, int nbins)
{
    const int T = tiles_for(nbins);
    const int64_t nseg = (npiv + kSeg - 1) / kSeg;
    return (size_t)(nseg > 0 ? nseg : 1) * (size_t)(m_max + 1) * (size_t)(T * (T + 1) / 2) * 256 * sizeof(double);
}

// G(u, v) of one segment, read from the tile holding min/max of (u, v).
__device__ __forceinline__ double gram_at(const double *seg_m, int T, int u, int v)
{
    if (u > v) { int t = u; u = v; v = t; }
    const int I = u >> 4, J = v >> 4;
    const int tp = I * T - I * (I - 1) / 2 + (J - I);
    return seg_m[(size_t)tp * 256 + (u & 15) * 16 + (v & 15)];
}

__global__ void k_gram_reduce(const double *part, int64_t nseg, int nmaps, int M1, int nb, int T, int ntp,
                              double *zeta, size_t z_stride)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int total = nmaps * M1 * nb * nb;
    if (t >= total) return;
    const int mm = t / (nb * nb), rem = t % (nb * nb), b1 = rem / nb, b2 = rem % nb;
    const int map = mm / M1, m = mm % M1;
    const int r1 = b1, r2 = b2, i1 = nb + b1, i2 = nb + b2;
    double rr = 0.0, ii = 0.0, ir = 0.0, ri = 0.0;
    for (int64_t s = 0; s < nseg; ++s) {
        const double *g = part + (size_t)((s * nmaps + map) * M1 + m) * ntp * 256;
        rr += gram_at(g, T, r1, r2);
        ii += gram_at(g, T, i1, i2);
        ir += gram_at(g, T, i1, r2);
        ri += gram_at(g, T, r1, i2);
    }
    double *z = zeta + map * z_stride + ((size_t)(m * nb + b1) * nb + b2) * 2;
    z[0] += rr + ii;
    z[1] += ir - ri;
}

// ---- LDS-staged pair contraction over pivot-minor multipoles --------------------------------
// G = sum_p v_p U1_p U2_p^T per (map, m): with U1 = U2 the Gram matrix of one field (only the
// tile pairs on or above the diagonal), else the full product of two fields (the multi-field
// estimator: Re zeta_m(b1, b2) = G(r1, r2) + G(i1, i2), Im zeta_m(b1, b2) = G(i1, r2) -
// G(r1, i2), i.e. sum_p v_p X1(b1) conj(X2(b2))).  One block per (pivot segment, map, m):
// tiles of kCrossKP pivots of the fields' 2nb rows of that m are staged in LDS as
// [pivot][row], consecutive pivots of a row on consecutive lanes (one contiguous run of the
// pivot-minor layout), and the waves run the 16 x 16 tile pairs out of LDS, so every
// multipole is read from memory once per launch; the next tile's loads are in flight
// during the current tile's MFMAs.  MFMA as in the pivot-major contraction below (split FP32
// operand on the mixed path), fixed-order FP64 sums.

struct PairArgs {
    const void *A1, *A2;  // [map][m+1][2][nb][ldA] multipoles of the b1 and b2 fields (Gram: A1 only)
    int64_t ldA;
    int64_t npiv;
    const double *v;      // pivot products w_p x_p of the pivot field
    size_t a_stride;      // elements between the maps' multipoles (Gram of several maps)
    size_t v_stride;      // elements between the maps' pivot products
    int nb, T, M1, nmaps;
    int npairs;           // tile pairs per (map, m): T^2, or T (T + 1) / 2 for a Gram matrix
    int ldr;              // LDS row length: the least >= 2 nb that is 17 mod 32 (conflict-free
                          // staging writes, 16 pivots of a row 17 banks apart; operand reads
                          // of the four pivot groups nearly so)
    double *part;         // [seg][map][m][npairs][256]
};

constexpr int kCrossKP = 32;  // pivots per LDS tile of the multi-field contraction (8 MFMA k-steps)

// NW waves per block, UPW tile pairs per wave, tile pairs blockIdx.y NW UPW onwards; each
// thread stages up to ROWS rows of both fields per tile (2 nb <= 16 T <= ROWS x 2 NW for
// every shape launched).  SYM: a Gram matrix of one field (A2 = A1; only the tile pairs on
// or above the diagonal, the others are their mirror).
template <bool F32, int NW, int UPW, int ROWS, bool SYM>
__global__ __launch_bounds__(NW * 64) void k_pair_lds(PairArgs c)
{
    typedef typename std::conditional<F32, float, double>::type E;
    constexpr int kThreads = NW * 64, kRows = ROWS;
    extern __shared__ __align__(16) unsigned char smem[];
    const int ldr = c.ldr;
    E *t1 = reinterpret_cast<E *>(smem);                          // [kCrossKP][ldr]
    E *t2 = SYM ? t1 : t1 + kCrossKP * ldr;                       // [kCrossKP][ldr]
    double *vt = reinterpret_cast<double *>(t1 + (SYM ? 1 : 2) * kCrossKP * ldr);  // [kCrossKP]
    const int64_t unit = blockIdx.x;  // (segment, map, m)
    const int m = (int)(unit % c.M1);
    const int map = (int)((unit / c.M1) % c.nmaps);
    const int64_t seg = unit / ((int64_t)c.M1 * c.nmaps);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int two_nb = 2 * c.nb, T = c.T;
    const size_t mo = (size_t)map * c.a_stride + (size_t)2 * m * c.nb * c.ldA;
    const E *src1 = static_cast<const E *>(c.A1) + mo;
    const E *src2 = static_cast<const E *>(SYM ? c.A1 : c.A2) + mo;
    const double *v = c.v + (size_t)map * c.v_stride;

    int ua[UPW], ub[UPW];
    v4d acc[UPW];
#pragma unroll
    for (int j = 0; j < UPW; ++j) {
        const int tp = (int)blockIdx.y * NW * UPW + wave + NW * j;
        acc[j] = v4d{0.0, 0.0, 0.0, 0.0};
        ua[j] = ub[j] = -1;
        if (tp < c.npairs) {
            int I = tp / T, J = tp % T;
            if constexpr (SYM) {
                int r = tp;
                I = 0;
                while (r >= T - I) { r -= T - I; ++I; }
                J = I + r;
            }
            ua[j] = I * 16 + row;
            ub[j] = J * 16 + row;
        }
    }
    const int64_t pbeg = seg * kSeg;
    const int64_t pend = min(c.npiv, pbeg + kSeg);
    // staging: thread -> (row u, pivot k), kCrossKP pivots of a row on consecutive lanes (one
    // contiguous run of the pivot-minor layout); the next tile's global loads are issued
    // before the current tile's MFMAs
    const int k = tid % kCrossKP, u0 = tid / kCrossKP, ustep = kThreads / kCrossKP;
    E a[kRows], b[kRows];
    auto fetch = [&](int64_t q0) {
        const bool kin = q0 + k < pend;
#pragma unroll
        for (int i = 0; i < kRows; ++i) {
            const int uu = u0 + i * ustep;
            const bool in = uu < two_nb && kin;
            a[i] = in ? src1[(size_t)uu * c.ldA + q0 + k] : E(0);
            if constexpr (!SYM) b[i] = in ? src2[(size_t)uu * c.ldA + q0 + k] : E(0);
        }
    };
    fetch(pbeg);
    for (int64_t p0 = pbeg; p0 < pend; p0 += kCrossKP) {
        const int np = (int)min((int64_t)kCrossKP, pend - p0);
        __syncthreads();  // the previous tile is consumed
#pragma unroll
        for (int i = 0; i < kRows; ++i) {
            const int uu = u0 + i * ustep;
            if (uu < two_nb) {
                t1[k * ldr + uu] = a[i];
                if constexpr (!SYM) t2[k * ldr + uu] = b[i];
            }
        }
        if (tid < kCrossKP) vt[tid] = tid < np ? v[p0 + tid] : 0.0;
        __syncthreads();
        if (p0 + kCrossKP < pend) fetch(p0 + kCrossKP);
#pragma unroll
        for (int h = 0; h < kCrossKP / 16; ++h) {
            double vk[4];
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) vk[ks] = vt[16 * h + 4 * ks + kq];
#pragma unroll
            for (int j = 0; j < UPW; ++j) {
                if (ua[j] < 0) continue;  // wave-uniform
                if constexpr (F32) {
                    // FP32 products over 16 pivots, then into the FP64 sum; the scaled operand
                    // v_p U1 is formed in FP64 and carried as FP32 hi + lo
                    v4f part = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        const int base = (16 * h + 4 * ks + kq) * ldr;
                        const float x1 = ua[j] < two_nb ? t1[base + ua[j]] : 0.0f;
                        const float x2 = ub[j] < two_nb ? t2[base + ub[j]] : 0.0f;
                        const double av = (double)x1 * vk[ks];
                        const float ahi = (float)av;
                        const float alo = (float)(av - (double)ahi);
                        part = __builtin_amdgcn_mfma_f32_16x16x4f32(ahi, x2, part, 0, 0, 0);
                        part = __builtin_amdgcn_mfma_f32_16x16x4f32(alo, x2, part, 0, 0, 0);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[j][q] += (double)part[q];
                } else {
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        const int base = (16 * h + 4 * ks + kq) * ldr;
                        const double x1 = ua[j] < two_nb ? t1[base + ua[j]] : 0.0;
                        const double x2 = ub[j] < two_nb ? t2[base + ub[j]] : 0.0;
                        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1 * vk[ks], x2, acc[j], 0, 0, 0);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < UPW; ++j) {
        if (ua[j] < 0) continue;
        const int tp = (int)blockIdx.y * NW * UPW + wave + NW * j;
        double *out = c.part + ((size_t)unit * (size_t)c.npairs + tp) * 256;
        // f64 16x16x4 result: register q of lane l is D[4q + l/16][l % 16];
        // f32 16x16x4 result: register q of lane l is D[4 (l/16) + q][l % 16]
#pragma unroll
        for (int q = 0; q < 4; ++q) out[(F32 ? 4 * kq + q : 4 * q + kq) * 16 + row] = acc[j][q];
    }
}

template <bool F32, int NW, int UPW, int ROWS, bool SYM>
static void launch_pair_lds(dim3 grid, size_t lds, const PairArgs &c, hipStream_t s)
{
    hipLaunchKernelGGL((k_pair_lds<F32, NW, UPW, ROWS, SYM>), grid, dim3(NW * 64), lds, s, c);
}

template <bool F32, bool SYM>
static void launch_pair_shape(dim3 grid, size_t lds, const PairArgs &c, hipStream_t s)
{
    // one tile pair per wave, as many waves as pairs up to T = 4 (6 or 9 waves at T = 3: 9
    // stage the 48 rows three per thread); beyond, groups of 16 pairs in blocks of their own
    // (grid.y), each staging the whole tile
    const int T = c.T;
    if (T <= 2) launch_pair_lds<F32, 4, 1, 4, SYM>(grid, lds, c, s);
    else if (T == 3 && SYM) launch_pair_lds<F32, 6, 1, 4, SYM>(grid, lds, c, s);
    else if (T == 3) launch_pair_lds<F32, 9, 1, 3, SYM>(grid, lds, c, s);
    else if (T == 4 && SYM) launch_pair_lds<F32, 10, 1, 4, SYM>(grid, lds, c, s);
    else launch_pair_lds<F32, 16, 1, 4, SYM>(dim3(grid.x, (unsigned)((c.npairs + 15) / 16)), lds, c, s);
}

// LDS-staged pair contraction over pivot-minor multipoles: one block per (segment, map, m)
static z3_status launch_pair(const PairArgs &c0, bool f32, bool sym, int64_t nseg, hipStream_t s)
{
    PairArgs c = c0;
    c.ldr = 2 * c.nb + ((17 - 2 * c.nb) % 32 + 32) % 32;
    const size_t tile = (size_t)kCrossKP * c.ldr * (f32 ? 4 : 8);
    const size_t lds = (sym ? 1 : 2) * (tile + 7) / 8 * 8 + kCrossKP * sizeof(double);
    int dev = 0, lds_max = 0;
    z3_status st = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st == Z3_OK)
        st = check_hip(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "LDS size");
    if (st != Z3_OK) return st;
    if (lds > (size_t)lds_max)
        return fail(Z3_ERR_UNSUPPORTED, "contraction of %d bins needs %zu bytes of LDS per block (%d)", c.nb, lds,
                    lds_max);
    const int64_t nblk = nseg * c.nmaps * c.M1;
    if (nblk > (int64_t)(UINT32_MAX / 1024))
        return fail(Z3_ERR_OVERFLOW, "contraction of %lld pivot segments x %d maps", (long long)nseg, c.nmaps);
    const dim3 grid((unsigned)nblk);
    if (f32) sym ? launch_pair_shape<true, true>(grid, lds, c, s) : launch_pair_shape<true, false>(grid, lds, c, s);
    else sym ? launch_pair_shape<false, true>(grid, lds, c, s) : launch_pair_shape<false, false>(grid, lds, c, s);
    return check_launch("k_pair_lds");
}

// ---- LDS-staged contraction of the pivot-major staging ------------------------------------
// One block of kGramWaves waves per (pivot segment, map).  Tiles of kGramKP pivots of the
// many-map kernel's pivot-major staging (one contiguous run of R = 2 (m_max + 1) rows per
// pivot and bin) are staged in LDS as [pivot][bin][row], runs on consecutive lanes.  Every
// wave then runs its (m, tile pair) units over the tile out of LDS, so each multipole is
// fetched once per block and the staging needs no transpose.
constexpr int kGramWaves = 8;
constexpr int kGramThreads = kGramWaves * 64;
constexpr int kGramKP = 16;                      // pivots per LDS tile (4 MFMA k-steps)
constexpr size_t kGramLdsMax = 64 * 1024 - 256;  // tile + pivot values

static size_t gram_tile_bytes(int nb, int R, bool f32)
{
    return ((size_t)kGramKP * nb * R * (f32 ? 4 : 8) + 15) / 16 * 16;
}

// units per wave: the smallest compiled bound covering M1 x (tile pairs) units, else 0 (more
// accumulators than a wave can hold at two waves per SIMD without spilling)
static int gram_upw(int nunits)
{
    for (int u : {5, 9})
        if (kGramWaves * u >= nunits) return u;
    return 0;
}

bool gram_lds_fits(int m_max, int nbins, int prec)
{
    const int T = tiles_for(nbins), ntp = T * (T + 1) / 2;
    const int R = 2 * (m_max + 1);
    return gram_upw((m_max + 1) * ntp) > 0 && R <= 64 &&
           gram_tile_bytes(nbins, R, prec == Z3_PREC_MIXED) + kGramKP * sizeof(double) <= kGramLdsMax;
}

// element (pivot p, bin b, row r) of map j at base + j map_stride + p sp + b sb + r sr
struct GramSrc {
    const void *base;
    int64_t sp, sb, sr;
    size_t map_stride;
};

struct GramArgs {
    GramSrc src;
    int64_t npiv;
    const double *v;
    size_t v_stride;
    int nb, R, T, ntp, M1, nmaps, nunits;
    int lpr_shift;       // PM staging: log2 of the lanes per (pivot, bin) run of R rows
    size_t tile_bytes;
    double *part;        // [seg][map][m][tile pair][256]
};

template <bool F32, int UPW>
__global__ __launch_bounds__(kGramThreads) void k_gram_lds(GramArgs g)
{
    typedef typename std::conditional<F32, float, double>::type T;
    extern __shared__ __align__(16) unsigned char smem[];
    T *tile = reinterpret_cast<T *>(smem);                          // [kGramKP][nb][R]
    double *vt = reinterpret_cast<double *>(smem + g.tile_bytes);   // [kGramKP]
    const int nb = g.nb, R = g.R, rowlen = nb * R;
    // blocks are dealt round-robin to the 8 XCDs: each XCD gets a contiguous run of
    // (segment, map) units, so blocks reading neighbouring maps' runs share its L2
    const int64_t nblk = gridDim.x, bi = blockIdx.x, per = nblk / 8;
    const int64_t unit = bi < per * 8 ? (bi % 8) * per + bi / 8 : bi;
    const int64_t seg = unit / g.nmaps;
    const int map = (int)(unit - seg * g.nmaps);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const T *src = static_cast<const T *>(g.src.base) + (size_t)map * g.src.map_stride;
    const double *v = g.v + (size_t)map * g.v_stride;

    // this wave's units (m, tile pair) and, for each, the offsets within one pivot's LDS row
    // of the A-operand and B-operand entries this lane supplies (-1: a padding row)
    int um[UPW], offa[UPW], offb[UPW];
    v4d acc[UPW];
#pragma unroll
    for (int j = 0; j < UPW; ++j) {
        const int uu = wave + kGramWaves * j;
        um[j] = offa[j] = offb[j] = -1;
        acc[j] = v4d{0.0, 0.0, 0.0, 0.0};
        if (uu < g.nunits) {
            const int m = uu / g.ntp;
            int r = uu - m * g.ntp, I = 0;
            while (r >= g.T - I) { r -= g.T - I; ++I; }
            const int J = I + r;
            const int ua = I * 16 + row, ub = J * 16 + row;
            um[j] = m;
            if (ua < 2 * nb) { const int c = ua >= nb; offa[j] = (ua - c * nb) * R + 2 * m + c; }
            if (ub < 2 * nb) { const int c = ub >= nb; offb[j] = (ub - c * nb) * R + 2 * m + c; }
        }
    }

    const int64_t pbeg = seg * kSeg;
    const int64_t pend = min(g.npiv, pbeg + kSeg);
    for (int64_t p0 = pbeg; p0 < pend; p0 += kGramKP) {
        const int np = (int)min((int64_t)kGramKP, pend - p0);
        __syncthreads();  // the previous tile is consumed
        // Each thread walks its elements (inner index b by `step`, wrapping into the outer
        // index) with incremental addresses, and issues the global loads of 8 elements
        // before it writes any of them to LDS, so their latencies overlap.
        // runs of R rows per (pivot, bin), contiguous in memory: lanes along the run
        const int step = kGramThreads >> g.lpr_shift;
        const int r = tid & ((1 << g.lpr_shift) - 1);
        const int kb0 = tid >> g.lpr_shift;
        int k = kb0 / nb, b = kb0 - k * nb;
        const T *ptr = src + (size_t)(p0 + k) * g.src.sp + (size_t)b * g.src.sb + r;
        int li = kb0 * R + r;
        const int64_t d_in = (int64_t)step * g.src.sb, d_wrap = g.src.sp - (int64_t)nb * g.src.sb;
        while (k < kGramKP) {
            T val[8];
            int at[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                at[i] = -1;
                if (k < kGramKP) {
                    if (r < R) at[i] = li;
                    val[i] = (k < np && r < R) ? *ptr : T(0);
                    b += step;
                    ptr += d_in;
                    li += step * R;
                    while (b >= nb) { b -= nb; ++k; ptr += d_wrap; }
                }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (at[i] >= 0) tile[at[i]] = val[i];
        }
        if (tid < kGramKP) vt[tid] = tid < np ? v[p0 + tid] : 0.0;
        __syncthreads();
        double vk[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) vk[ks] = vt[4 * ks + kq];
#pragma unroll
        for (int j = 0; j < UPW; ++j) {
            if (um[j] < 0) continue;  // wave-uniform
            if constexpr (F32) {
                // FP32 products and sums over the tile's pivots, then into the FP64 sum; the
                // scaled operand v_p U_i is formed in FP64 and carried as FP32 hi + lo
                v4f part = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int base = (4 * ks + kq) * rowlen;
                    const float ua = offa[j] >= 0 ? tile[base + offa[j]] : 0.0f;
                    const float ub = offb[j] >= 0 ? tile[base + offb[j]] : 0.0f;
                    const double av = (double)ua * vk[ks];
                    const float ahi = (float)av;
                    const float alo = (float)(av - (double)ahi);
                    part = __builtin_amdgcn_mfma_f32_16x16x4f32(ahi, ub, part, 0, 0, 0);
                    part = __builtin_amdgcn_mfma_f32_16x16x4f32(alo, ub, part, 0, 0, 0);
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) acc[j][k] += (double)part[k];
            } else {
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int base = (4 * ks + kq) * rowlen;
                    const double ua = offa[j] >= 0 ? tile[base + offa[j]] : 0.0;
                    const double ub = offb[j] >= 0 ? tile[base + offb[j]] : 0.0;
                    acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua * vk[ks], ub, acc[j], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < UPW; ++j) {
        if (um[j] < 0) continue;
        const int tp = wave + kGramWaves * j - um[j] * g.ntp;
        double *out = g.part + ((((size_t)seg * g.nmaps + map) * g.M1 + um[j]) * g.ntp + tp) * 256;
        // f64 16x16x4 result: register k of lane l is D[4k + l/16][l % 16];
        // f32 16x16x4 result: register k of lane l is D[4 (l/16) + k][l % 16]
#pragma unroll
        for (int k = 0; k < 4; ++k) out[(F32 ? 4 * kq + k : 4 * k + kq) * 16 + row] = acc[j][k];
    }
}

template <bool F32>
static void launch_gram_lds(int upw, dim3 grid, size_t lds, const GramArgs &g, hipStream_t s)
{
    if (upw == 5) hipLaunchKernelGGL((k_gram_lds<F32, 5>), grid, dim3(kGramThreads), lds, s, g);
    else hipLaunchKernelGGL((k_gram_lds<F32, 9>), grid, dim3(kGramThreads), lds, s, g);
}

static z3_status contract_src(int64_t npiv, int m_max, int nbins, int prec, int nmaps, const GramSrc &src, bool pm,
                              const double *piv_v, size_t v_stride, double *zeta, size_t z_stride, void *partials,
                              size_t partial_bytes, hipStream_t s)
{
    if (npiv <= 0 || nmaps <= 0) return Z3_OK;
    const int T = tiles_for(nbins), ntp = T * (T + 1) / 2;
    const int64_t nseg = (npiv + kSeg - 1) / kSeg;
    if (contract_partial_bytes(npiv, m_max, nbins) * (size_t)nmaps > partial_bytes)
        return fail(Z3_ERR_INVALID_ARG, "contraction workspace too small");
    if (nseg > 65535) return fail(Z3_ERR_OVERFLOW, "too many pivots for one contraction (%lld)", (long long)npiv);
    if ((int64_t)nmaps * (m_max + 1) > 65535) return fail(Z3_ERR_OVERFLOW, "too many maps for one contraction");
    const bool f32 = prec == Z3_PREC_MIXED;
    z3_status st;
    if (pm) {
        if (!gram_lds_fits(m_max, nbins, prec))
            return fail(Z3_ERR_UNSUPPORTED, "pivot-major contraction for m_max=%d, %d bins", m_max, nbins);
        // one block per (segment, map): the dispatch stays below 2^32 work-items
        if (nseg * nmaps > (int64_t)(UINT32_MAX / kGramThreads))
            return fail(Z3_ERR_OVERFLOW, "contraction of %lld pivots x %d maps in one launch", (long long)npiv, nmaps);
        GramArgs g;
        g.src = src;
        g.npiv = npiv;
        g.v = piv_v;
        g.v_stride = v_stride;
        g.nb = nbins;
        g.R = 2 * (m_max + 1);
        g.T = T;
        g.ntp = ntp;
        g.M1 = m_max + 1;
        g.nmaps = nmaps;
        g.nunits = (m_max + 1) * ntp;
        g.lpr_shift = g.R <= 32 ? 5 : 6;
        g.tile_bytes = gram_tile_bytes(nbins, g.R, f32);
        g.part = static_cast<double *>(partials);
        const int upw = gram_upw(g.nunits);
        const dim3 grid((unsigned)(nseg * nmaps));
        const size_t lds = g.tile_bytes + kGramKP * sizeof(double);
        if (f32) launch_gram_lds<true>(upw, grid, lds, g, s);
        else launch_gram_lds<false>(upw, grid, lds, g, s);
        st = check_launch("k_gram_lds");
    } else {
        PairArgs c = {};
        c.A1 = src.base;
        c.ldA = src.sb;
        c.npiv = npiv;
        c.v = piv_v;
        c.a_stride = src.map_stride;
        c.v_stride = v_stride;
        c.nb = nbins;
        c.T = T;
        c.M1 = m_max + 1;
        c.nmaps = nmaps;
        c.npairs = ntp;
        c.part = static_cast<double *>(partials);
        st = launch_pair(c, f32, true, nseg, s);
    }
    if (st != Z3_OK) return st;
    const int total = nmaps * (m_max + 1) * nbins * nbins;
    hipLaunchKernelGGL(k_gram_reduce, dim3((total + 127) / 128), dim3(128), 0, s,
                       static_cast<const double *>(partials), nseg, nmaps, m_max + 1, nbins, T, ntp, zeta, z_stride);
    return check_launch("k_gram_reduce");
}

z3_status launch_contract_maps(int64_t npiv, int m_max, int nbins, int prec, int nmaps, const void *A, int64_t ldA,
                               size_t a_stride, const double *piv_v, size_t v_stride, double *zeta, size_t z_stride,
                               void *partials, size_t partial_bytes, hipStream_t s)
{
    const GramSrc src{A, 1, ldA, (int64_t)nbins * ldA, a_stride};
    return contract_src(npiv, m_max, nbins, prec, nmaps, src, false, piv_v, v_stride, zeta, z_stride, partials,
                        partial_bytes, s);
}

z3_status launch_contract_staged(int64_t npiv, int m_max, int nbins, int prec, int nmaps, const void *stage,
                                 const double *piv_v, size_t v_stride, double *zeta, size_t z_stride, void *partials,
                                 size_t partial_bytes, hipStream_t s)
{
    const int64_t R = 2 * (m_max + 1);
    const GramSrc src{stage, (int64_t)nbins * nmaps * R, (int64_t)nmaps * R, 1, (size_t)R};
    return contract_src(npiv, m_max, nbins, prec, nmaps, src, true, piv_v, v_stride, zeta, z_stride, partials,
                        partial_bytes, s);
}

z3_status launch_contract(int64_t npiv, int m_max, int nbins, int prec, const void *A, int64_t ldA,
                          const double *piv_v, double *zeta, void *partials, size_t partial_bytes,
                          hipStream_t s)
{
    return launch_contract_maps(npiv, m_max, nbins, prec, 1, A, ldA, 0, piv_v, 0, zeta, 0, partials, partial_bytes, s);
}

__device__ __forceinline__ double cross_at(const double *seg_m, int T, int u, int v)
{
    return seg_m[(size_t)((u >> 4) * T + (v >> 4)) * 256 + (u & 15) * 16 + (v & 15)];
}

__global__ void k_cross_reduce(const double *part, int64_t nseg, int M1, int nb, int T, double *zeta)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M1 * nb * nb) return;
    const int m = t / (nb * nb), rem = t % (nb * nb), b1 = rem / nb, b2 = rem % nb;
    const int r1 = b1, r2 = b2, i1 = nb + b1, i2 = nb + b2;
    double rr = 0.0, ii = 0.0, ir = 0.0, ri = 0.0;
    for (int64_t s = 0; s < nseg; ++s) {
        const double *g = part + (size_t)(s * M1 + m) * (size_t)(T * T) * 256;
        rr += cross_at(g, T, r1, r2);
        ii += cross_at(g, T, i1, i2);
        ir += cross_at(g, T, i1, r2);
        ri += cross_at(g, T, r1, i2);
    }
    double *z = zeta + ((size_t)(m * nb + b1) * nb + b2) * 2;
    z[0] += rr + ii;
    z[1] += ir - ri;
}

size_t cross_partial_bytes(int64_t npiv, int m_max, int nbins)
{
    const int T = tiles_for(nbins);
    const int64_t nseg = (npiv + kSeg - 1) / kSeg;
    return (size_t)(nseg > 0 ? nseg : 1) * (size_t)(m_max + 1) * (size_t)(T * T) * 256 * sizeof(double);
}

z3_status launch_contract_cross(int64_t npiv, int m_max, int nbins, int prec, const void *A1, const void *A2,
                                int64_t ldA, const double *piv_v, double *zeta, void *partials,
                                size_t partial_bytes, hipStream_t s)
{
    if (npiv <= 0) return Z3_OK;
    const int T = tiles_for(nbins);
    const int64_t nseg = (npiv + kSeg - 1) / kSeg;
    if (partial_bytes < cross_partial_bytes(npiv, m_max, nbins))
        return fail(Z3_ERR_INVALID_ARG, "multi-field contraction: partial buffer too small");
    PairArgs c = {};
    c.A1 = A1;
    c.A2 = A2;
    c.ldA = ldA;
    c.npiv = npiv;
    c.v = piv_v;
    c.nb = nbins;
    c.T = T;
    c.M1 = m_max + 1;
    c.nmaps = 1;
    c.npairs = T * T;
    c.part = static_cast<double *>(partials);
    z3_status st = launch_pair(c, prec == Z3_PREC_MIXED, false, nseg, s);
    if (st != Z3_OK) return st;
    const int total = (m_max + 1) * nbins * nbins;
    hipLaunchKernelGGL(k_cross_reduce, dim3((total + 127) / 128), dim3(128), 0, s,
                       static_cast<const double *>(partials), nseg, m_max + 1, nbins, T, zeta);
    return check_launch("k_cross_reduce");
}

// ---- sum of pivot weights (fixed order) ------------------------------------------------

__global__ void k_sum_partials(const double *w, int64_t n, int64_t per_block, double *partial)
{
    __shared__ double sh[256];
    const int64_t beg = (int64_t)blockIdx.x * per_block;
    const int64_t end = min(n, beg + per_block);
    double acc = 0.0;
    for (int64_t i = beg + threadIdx.x; i < end; i += 256) acc += w[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_sum_final(const double *partial, int nblk, double *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double acc = 0.0;
        for (int b = 0; b < nblk; ++b) acc += partial[b];
        out[0] += acc;
    }
}

z3_status launch_weight_sum(const double *w, int64_t n, double *out, hipStream_t s)
{
    int64_t want = (n + 4095) / 4096;
    int nblk = (int)(want < 1024 ? want : 1024);
    if (nblk < 1) nblk = 1;
    const int64_t per = (n + nblk - 1) / nblk;
    void *part = nullptr;
    z3_status st = scratch_alloc(&part, nblk * sizeof(double), s);
    if (st != Z3_OK) return st;
    double *partial = static_cast<double *>(part);
    hipLaunchKernelGGL(k_sum_partials, dim3(nblk), dim3(256), 0, s, w, n, per, partial);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(64), 0, s, partial, nblk, out);
    st = check_launch("k_sum");
    scratch_free(part, s);
    return st;
}

__global__ void k_pivot_values(const double *w, const double *x, int64_t n, double *v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = w ? w[i] * x[i] : x[i];
}

z3_status launch_pivot_values(const double *w, const double *x, int64_t n, double *v, hipStream_t s)
{
    if (n <= 0) return Z3_OK;
    hipLaunchKernelGGL(k_pivot_values, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, x, n, v);
    return check_launch("k_pivot_values");
}

__global__ void k_fill_value(double *p, int64_t n, double value)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

// Fills with a kernel rather than a memset, so that the call can sit in a captured graph.
z3_status launch_fill(double *p, int64_t n, double value, hipStream_t s)
{
    if (n <= 0) return Z3_OK;
    hipLaunchKernelGGL(k_fill_value, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, value);
    return check_launch("k_fill_value");
}

__global__ void k_add_scalar(double *out, double value)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] += value;
}

z3_status launch_add_scalar(double *out, double value, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_scalar, dim3(1), dim3(64), 0, s, out, value);
    return check_launch("k_add_scalar");
}

__global__ void k_finalize(double *zeta, int64_t count, const double *sum_w)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // an empty pivot set (sum of weights 0) leaves the (zero) sums unchanged
    if (i < count && sum_w[0] != 0.0) zeta[i] /= sum_w[0];
}

z3_status launch_finalize(int nmaps, int m_max, int nbins, double *zeta, const double *sum_w, hipStream_t s)
{
    const int64_t count = (int64_t)nmaps * (m_max + 1) * nbins * nbins * 2;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, zeta, count, sum_w);
    return check_launch("k_finalize");
}

// Removal of the k = j terms: one block per bin adds the bin's column of the per-wave
// sums v_p Q / W^2 in a fixed order and subtracts the total from Re zeta_m(b, b) for every
// m (those terms are real and the same for every m).
__global__ void k_self_subtract(const double *part, int64_t nw, int nb, int M, double *zeta)
{
    __shared__ double sh[256];
    const int b = blockIdx.x;
    double acc = 0.0;
    for (int64_t w = threadIdx.x; w < nw; w += 256) acc += part[w * nb + b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if ((int)threadIdx.x <= M) zeta[(((size_t)threadIdx.x * nb + b) * nb + b) * 2] -= sh[0];
}

z3_status launch_self_subtract(const double *part, int64_t nw, int m_max, int nbins, double *zeta, hipStream_t s)
{
    if (nw <= 0) return Z3_OK;
    hipLaunchKernelGGL(k_self_subtract, dim3(nbins), dim3(256), 0, s, part, nw, nbins, m_max, zeta);
    return check_launch("k_self_subtract");
}

// zeta(b1, b2, phi) = Re zeta_0 + 2 sum_{m>=1} (Re zeta_m cos(m phi) - Im zeta_m sin(m phi))
__global__ void k_resum(int M, int nb, const double *zeta, int nphi, const double *phi, double *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nb * nb * nphi) return;
    const int k = (int)(t % nphi);
    const int64_t bb = t / nphi;
    const double ph = phi[k];
    double acc = zeta[bb * 2];
    for (int m = 1; m <= M; ++m) {
        const double *z = zeta + ((size_t)m * nb * nb + bb) * 2;
        double sm, cm;
        sincos(m * ph, &sm, &cm);
        acc += 2.0 * (z[0] * cm - z[1] * sm);
    }
    out[t] = acc;
}

z3_status launch_resum(int m_max, int nbins, const double *zeta, int nphi, const double *phi, double *out,
                       hipStream_t s)
{
    const int64_t total = (int64_t)nbins * nbins * nphi;
    hipLaunchKernelGGL(k_resum, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, m_max, nbins, zeta, nphi,
                       phi, out);
    return check_launch("k_resum");
}

}  // namespace z3
