// FFTLog evaluation of the line-of-sight integrals of the modelling appendix ("FFTLog for the
// line-of-sight integral"): the functions A_0, A_1, A_2 of a batch of models sharing P_L(k)
// and the angle grid, each with its own line-of-sight kernel F(chi) = q_A q_B q_C D_+^4.
//
//   c_s   = W_s k_min^{-nu - i eta_s} (1/N) sum_l P(k_l) (k_l/k_min)^{-nu} e^{-2 pi i s l/N}
//           (eqs. pklfft, pklfft_eta, cm; s = -N/2..N/2; one set per bias nu)
//   g(a)  = 2^{mt+a-1} Gamma((1+mt+a+n)/2) / (pi Gamma((1-a-mt+n)/2)),   a_s = 1 + nu + i eta_s
//           (the closed-form k integral of the appendix)
//   U_{is}= c_s g(a_s) theta_i^{-(1 + a_s + mt)}                         per factor (n, mt, nu)
//   A_{s1 s2} = int dchi F(chi) chi^{-a_s1 - a_s2 - 2}                  (trapezoid in ln chi)
//   I     = U1 A U2^T,   A_0 = I^{(0,0)}_{(0,0)},  A_1 = I^{(1,1)}_{(1,-1)} + transpose,
//           A_2 = I^{(2,0)}_{(2,0)}
//
// Two structural facts shape the evaluation:
//  * eta_s is linear in s (eta_s = s deta), so chi^{-a_s1 - a_s2} = chi^{-(2 + nu1 + nu2)}
//    e^{-i (s1 + s2) deta ln chi}: the stored matrix is a Hankel matrix, A_{s1 s2} = h(s1 + s2)
//    with only 2N + 1 distinct entries
//        h(t) = sum_j d_j chi_j^{-(2 + nu1 + nu2)} e^{-i t deta ln chi_j},   t = -N..N,
//    d_j the trapezoid weights in ln chi times F chi^{-1}; h(-t) = conj h(t).
//  * P is real, so c_{-s} = conj c_s, and with real nu every factor obeys U_{i,-s} = conj U_{is}:
//    the terms (s1, s2) and (-s1, -s2) are conjugate, I is real, and
//        I = Re sum_{s1 >= 0} omega_s1 sum_{s2} U1_{i s1} h(s1 + s2) U2_{j s2},
//    omega_0 = 1, omega_{s1 > 0} = 2 (the s1 = 0 column of U1 is real).
// So the library forms h for t >= 0 for every model and factor pair as one real-by-complex
// product over chi (E_{jt} = e^{-i t deta ln chi_j}, shared by all models), mirrors it to
// t < 0, then UA = (omega U1)_{s1 >= 0} H (H read straight from h) and Re(UA U2^T): complex
// FP64 matrix products on v_mfma_f64_16x16x4f64 through one strided batched kernel, 8 (N+1)
// (N/2+1) ntheta + 4 ntheta^2 (N+1) flop per function and model in place of the dense
// evaluation's 8 (N+1)^2 (nchi + ntheta) + 8 ntheta^2 (N+1).  The coefficient DFT and the Gamma
// ratios (complex log-Gamma: upward recurrence to Re z >= 12, then Stirling's series) run one
// wave per coefficient; the operands are elementwise kernels.
#include <type_traits>

#include "z3_internal.h"

namespace z3 {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

__device__ __forceinline__ double2 cexp(double2 z)
{
    double s, c;
    sincos(z.y, &s, &c);
    const double e = exp(z.x);
    return make_double2(e * c, e * s);
}

__device__ __forceinline__ double2 clog(double2 z) { return make_double2(0.5 * log(z.x * z.x + z.y * z.y), atan2(z.y, z.x)); }

__device__ __forceinline__ double2 cdiv(double2 a, double2 b)
{
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// log Gamma(z) for complex z away from the poles, up to a multiple of 2 pi i in the imaginary
// part (only exp of differences is used).  Upward recurrence log Gamma(z) = log Gamma(z + K) -
// log prod_{j<K} (z + j) until Re(z + K) >= 12 (the product kept as one complex number, one
// logarithm at the end), then Stirling's series with Bernoulli terms B_{2k} / (2k (2k-1)
// z^{2k-1}), k = 1..8.
__device__ double2 clgamma(double2 z)
{
    double2 prod = make_double2(1.0, 0.0);
    bool shifted = false;
    while (z.x < 12.0) {
        prod = cmul(prod, z);
        z.x += 1.0;
        shifted = true;
    }
    const double2 shift = shifted ? clog(prod) : make_double2(0.0, 0.0);
    const double2 lz = clog(z);
    const double2 zh = make_double2(z.x - 0.5, z.y);
    double2 r = cmul(zh, lz);
    r.x += -z.x + 0.91893853320467274178;  // ln(2 pi) / 2
    r.y += -z.y;
    const double2 iz = cdiv(make_double2(1.0, 0.0), z);
    const double2 iz2 = cmul(iz, iz);
    const double b[8] = {1.0 / 12.0, -1.0 / 360.0, 1.0 / 1260.0, -1.0 / 1680.0, 1.0 / 1188.0, -691.0 / 360360.0,
                         1.0 / 156.0, -3617.0 / 122400.0};
    double2 t = iz, s = make_double2(0.0, 0.0);
    for (int k = 0; k < 8; ++k) {
        s.x += b[k] * t.x;
        s.y += b[k] * t.y;
        t = cmul(t, iz2);
    }
    return make_double2(r.x + s.x - shift.x, r.y + s.y - shift.y);
}

struct FactorSpec {
    int n, mt;
    double nu;
};

struct FftlogArgs {
    int N;                    // samples of P (even); Ns = N + 1 coefficients s = 0..N (m = s - N/2)
    int Ns, ld, ldw, ldh;     // padded lengths: s (ld), s1 >= 0 half (ldw), t >= 0 half (ldh)
    const double *Pk;
    double k_min, k_max;
    FactorSpec f[4];          // (0,0), (1,1), (1,-1), (2,0)
    int nchi;
    double chi_min, dlnchi;
    int T;
    const double *theta;
    double2 *cg;              // [4][ld]: c_s g(a_s)
    double2 *a;               // [4][ld]: a_s
    double2 *U;               // [4][T][ld]
    double2 *Uw;              // [4][T][ldw]: omega_m U[.][N/2 + m], m = 0..N/2
    double2 *E;               // [nchi][ldh]: e^{-i t deta ln chi_j}, t = 0..N
};

__device__ __forceinline__ double fftlog_deta(int N, double k_min, double k_max)
{
    return (double)(N - 1) / N * 2.0 * kPi / log(k_max / k_min);
}

// c_s (eq. cm), a_s and c_s g(a_s): one wave per (s, factor), the DFT over l split across lanes
__global__ __launch_bounds__(64) void k_fftlog_coeffs(FftlogArgs g)
{
    const int s = blockIdx.x, f = blockIdx.y, lane = threadIdx.x;
    const int N = g.N, m = s - N / 2;
    const double nu = g.f[f].nu;
    const double L = log(g.k_max / g.k_min), dl = L / (N - 1);
    const int mm = ((m % N) + N) % N;
    double re = 0.0, im = 0.0;
    for (int l = lane; l < N; l += 64) {
        const double v = g.Pk[l] * exp(-nu * dl * l);
        const int q = (int)(((unsigned)mm * (unsigned)l) % (unsigned)N);  // exact residue (< 2^24 product)
        double sn, cs;
        sincospi(2.0 * q / N, &sn, &cs);
        re += v * cs;
        im -= v * sn;
    }
    for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o, 64);
        im += __shfl_xor(im, o, 64);
    }
    if (lane > 1) return;
    const double eta = fftlog_deta(N, g.k_min, g.k_max) * m;
    const double2 a = make_double2(1.0 + nu, eta);
    const int n = g.f[f].n, mt = g.f[f].mt;
    // lane 0: log Gamma((1 + mt + a + n)/2); lane 1: log Gamma((1 - a - mt + n)/2)
    const double2 lg = clgamma(lane == 0 ? make_double2(0.5 * (1.0 + mt + a.x + n), 0.5 * a.y)
                                         : make_double2(0.5 * (1.0 - a.x - mt + n), -0.5 * a.y));
    const double2 l1 = make_double2(__shfl(lg.x, 0, 64), __shfl(lg.y, 0, 64));
    const double2 l2 = make_double2(__shfl(lg.x, 1, 64), __shfl(lg.y, 1, 64));
    if (lane) return;
    const double w = (s == 0 || s == N) ? 0.5 : 1.0;
    const double2 pre = cexp(make_double2(-nu * log(g.k_min), -eta * log(g.k_min)));
    const double2 c = cmul(pre, make_double2(w * re / N, w * im / N));
    const double ln2 = 0.69314718055994530942;
    const double2 gl = make_double2((mt + a.x - 1.0) * ln2 + l1.x - l2.x, a.y * ln2 + l1.y - l2.y);
    double2 cg = cmul(c, cexp(gl));
    cg.x /= kPi;
    cg.y /= kPi;
    g.cg[(size_t)f * g.ld + s] = cg;
    g.a[(size_t)f * g.ld + s] = a;
}

// U[f][i][s] = c_s g(a_s) theta_i^{-(1 + a_s + mt)} and its weighted upper half Uw; one thread
// per (factor, angle, s < Ns)
__global__ void k_fftlog_operands(FftlogArgs g)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)4 * g.T * g.Ns) return;
    const int s = (int)(t % g.Ns), i = (int)((t / g.Ns) % g.T), f = (int)(t / ((int64_t)g.Ns * g.T));
    const int mt = g.f[f].mt;
    const double2 cg = g.cg[(size_t)f * g.ld + s], a = g.a[(size_t)f * g.ld + s];
    const double lt = log(g.theta[i]);
    const double2 u = cmul(cg, cexp(make_double2(-(1.0 + a.x + mt) * lt, -a.y * lt)));
    g.U[((size_t)f * g.T + i) * g.ld + s] = u;
    const int m = s - g.N / 2;
    if (m >= 0) {
        const double om = m ? 2.0 : 1.0;
        g.Uw[((size_t)f * g.T + i) * g.ldw + m] = make_double2(om * u.x, om * u.y);
    }
}

// E[j][t] = e^{-i t deta ln chi_j}, t = 0..N
__global__ void k_fftlog_phases(FftlogArgs g)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)g.nchi * (g.N + 1)) return;
    const int t = (int)(e % (g.N + 1)), j = (int)(e / (g.N + 1));
    const double lc = log(g.chi_min) + j * g.dlnchi;
    double sn, cs;
    sincos(-(double)t * fftlog_deta(g.N, g.k_min, g.k_max) * lc, &sn, &cs);
    g.E[(size_t)j * g.ldh + t] = make_double2(cs, sn);
}

// weights of each (factor pair q, model b): D[q][b][j] = w_j F_b(chi_j) chi_j^{-1} chi_j^{-(2 + nu1 + nu2)}
// (w_j the trapezoid weights in ln chi)
__global__ void k_fftlog_weights(const double *F, int nchi, int nmodels, double chi_min, double dlnchi,
                                 double3 nusum, double *D)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nchi * nmodels * 3) return;
    const int j = (int)(t % nchi);
    const int q = (int)(t / ((int64_t)nchi * nmodels));
    const int64_t bj = t % ((int64_t)nchi * nmodels);
    const double lc = log(chi_min) + j * dlnchi;
    const double w = (j == 0 || j == nchi - 1) ? 0.5 * dlnchi : dlnchi;
    const double e = q == 0 ? nusum.x : q == 1 ? nusum.y : nusum.z;
    D[t] = w * F[bj] * exp(-(3.0 + e) * lc);
}

// Batched FP64 matrix product C[b] = A[b] B[b], elements addressed by strides (a Hankel operand
// H_{kj} = h[k + j] is b_k = b_j = 1).  A is complex; by TAG:
//   1: B real, C complex, and each row i of C also written, conjugated, at row -i (the mirror
//      h(-t) = conj h(t))
//   2: B and C complex
//   3: B complex, only Re C computed and stored (as double)
// Each wave computes a (16 RM) x 16 tile of C (RM 16 x 16 MFMA tiles sharing one B fragment).
// With KSPLIT the block's four waves share one tile and split the k range (k-steps of 8, wave w
// takes steps w, w + 4, ...; partial sums added through LDS in a fixed order, so results are
// deterministic): for products with few output tiles and a long k range.  Without it the four
// waves take four neighbouring column tiles.  The fragments of the next k-step are loaded
// before the current step's MFMAs.  Operand lane
// layout of v_mfma_f64_16x16x4f64: A row / B column = lane & 15, k = lane >> 4.
struct CGemm {
    const double2 *A;
    int64_t a_i, a_k, a_b;
    const void *B;
    int64_t b_k, b_j, b_b;
    void *C;
    int64_t c_i, c_j, c_b;
    int M, N, K;
};

template <int TAG, int RM, bool KSPLIT>
__global__ __launch_bounds__(256) void k_cgemm(CGemm g)
{
    constexpr bool BREAL = TAG == 1, CREAL = TAG == 3;
    typedef typename std::conditional<BREAL, double, double2>::type BT;
    __shared__ double red[3][8][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j0 = KSPLIT ? blockIdx.x * 16 : (blockIdx.x * 4 + w) * 16;
    if (!KSPLIT && j0 >= g.N) return;  // no barrier in this mode
    const int i0 = blockIdx.y * 16 * RM, b = blockIdx.z;
    const int r = lane & 15, q = lane >> 4;
    const int nrm = min(RM, (g.M - i0 + 15) / 16);  // block-uniform count of live row tiles
    const double2 *A = g.A + (size_t)b * g.a_b;
    const BT *B = static_cast<const BT *>(g.B) + (size_t)b * g.b_b;
    const int jb = j0 + r;
    const bool jin = jb < g.N;

    // per-lane row pointers of A and column pointer of B; k offsets stay 32-bit (k a_k, k b_k
    // < 2^31 for every product launched)
    const double2 *Ar[RM];
    bool rok[RM];
#pragma unroll
    for (int u = 0; u < RM; ++u) {
        const int i = i0 + 16 * u + r;
        rok[u] = u < nrm && i < g.M;
        Ar[u] = A + (rok[u] ? (size_t)i * g.a_i : 0);
    }
    const BT *Bc = B + (jin ? (size_t)jb * g.b_j : 0);
    const int ak = (int)g.a_k, bk = (int)g.b_k;
    auto load = [&](int k, double2 (&av)[RM], BT &bv) {
        const bool kin = k < g.K;
#pragma unroll
        for (int u = 0; u < RM; ++u) av[u] = (kin && rok[u]) ? Ar[u][k * ak] : make_double2(0.0, 0.0);
        if constexpr (BREAL)
            bv = (kin && jin) ? Bc[k * bk] : 0.0;
        else
            bv = (kin && jin) ? Bc[k * bk] : make_double2(0.0, 0.0);
    };
    v4d re[RM], im[RM];
#pragma unroll
    for (int u = 0; u < RM; ++u) {
        re[u] = v4d{0.0, 0.0, 0.0, 0.0};
        im[u] = v4d{0.0, 0.0, 0.0, 0.0};
    }
    auto step = [&](const double2 (&av)[RM], const BT &bv) {
        if constexpr (BREAL) {
#pragma unroll
            for (int u = 0; u < RM; ++u)
                if (u < nrm) re[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].x, bv, re[u], 0, 0, 0);
#pragma unroll
            for (int u = 0; u < RM; ++u)
                if (u < nrm) im[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].y, bv, im[u], 0, 0, 0);
        } else if constexpr (CREAL) {
#pragma unroll
            for (int u = 0; u < RM; ++u)
                if (u < nrm) re[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].x, bv.x, re[u], 0, 0, 0);
#pragma unroll
            for (int u = 0; u < RM; ++u)
                if (u < nrm) re[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[u].y, bv.y, re[u], 0, 0, 0);
        } else {
#pragma unroll
            for (int u = 0; u < RM; ++u)
                if (u < nrm) {
                    re[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].x, bv.x, re[u], 0, 0, 0);
                    im[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].x, bv.y, im[u], 0, 0, 0);
                }
#pragma unroll
            for (int u = 0; u < RM; ++u)
                if (u < nrm) {
                    re[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[u].y, bv.y, re[u], 0, 0, 0);
                    im[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].y, bv.x, im[u], 0, 0, 0);
                }
        }
    };
    double2 a0[RM], a1[RM];
    BT b0, b1;
    constexpr int kstride = KSPLIT ? 32 : 8;
    int k0 = KSPLIT ? 8 * w : 0;
    load(k0 + q, a0, b0);
    for (; k0 < g.K; k0 += kstride) {
        load(k0 + 4 + q, a1, b1);
        step(a0, b0);
        if (k0 + 4 >= g.K) break;
        load(k0 + kstride + q, a0, b0);
        step(a1, b1);
    }
    // partial sums of waves 1..3 added into wave 0's, one row tile at a time
    for (int u = 0; KSPLIT && u < RM; ++u) {
        if (u >= nrm) break;
        if (w > 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                red[w - 1][k][lane] = re[u][k];
                red[w - 1][4 + k][lane] = im[u][k];
            }
        }
        __syncthreads();
        if (w == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                re[u][k] = ((re[u][k] + red[0][k][lane]) + red[1][k][lane]) + red[2][k][lane];
                im[u][k] = ((im[u][k] + red[0][4 + k][lane]) + red[1][4 + k][lane]) + red[2][4 + k][lane];
            }
        }
        __syncthreads();
    }
    if ((KSPLIT && w > 0) || !jin) return;
    // v_mfma_f64_16x16x4f64 result layout: register k of lane l holds D[4k + l/16][l % 16]
#pragma unroll
    for (int u = 0; u < RM; ++u) {
        if (u >= nrm) break;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = i0 + 16 * u + 4 * k + q;
            if (i >= g.M) continue;
            const int64_t o = (size_t)b * g.c_b + i * g.c_i + jb * g.c_j;
            if constexpr (CREAL) {
                static_cast<double *>(g.C)[o] = re[u][k];
            } else {
                double2 *C = static_cast<double2 *>(g.C);
                C[o] = make_double2(re[u][k], im[u][k]);
                if constexpr (TAG == 1) C[o - 2 * i * g.c_i] = make_double2(re[u][k], -im[u][k]);
            }
        }
    }
}

template <int TAG, int RM, bool KSPLIT>
static z3_status cgemm(const CGemm &g, int batch, hipStream_t s)
{
    const int cols = KSPLIT ? 16 : 64;
    const dim3 grid((unsigned)((g.N + cols - 1) / cols), (unsigned)((g.M + 16 * RM - 1) / (16 * RM)),
                    (unsigned)batch);
    hipEvent_t ev0 = nullptr;
    if (TAG == 2) profile_begin(s, &ev0);
    hipLaunchKernelGGL((k_cgemm<TAG, RM, KSPLIT>), grid, dim3(256), 0, s, g);
    if (TAG == 2) profile_end(s, ev0);
    return check_launch("k_cgemm");
}

// out[b][0] = I0, out[b][1] = I1 + I1^T, out[b][2] = I2 (I real, [b][3][T][T])
__global__ void k_fftlog_out(const double *I, int T, int nmodels, double *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)T * T;
    if (t >= per * 3 * nmodels) return;
    const int64_t b = t / (3 * per), rem = t % (3 * per);
    const int p = (int)(rem / per), ij = (int)(rem % per), i = ij / T, j = ij % T;
    const double *Ib = I + (size_t)(b * 3 + p) * per;
    double v = Ib[ij];
    if (p == 1) v += Ib[(size_t)j * T + i];
    out[t] = v;
}

struct FftlogLayout {
    size_t ld, ldw, ldh, ldt;
};

static FftlogLayout fftlog_layout(int N)
{
    auto up16 = [](size_t v) { return (v + 15) / 16 * 16; };
    return FftlogLayout{up16((size_t)N + 1), up16((size_t)N / 2 + 1), up16((size_t)N + 1), up16(2 * (size_t)N + 1)};
}

size_t fftlog_workspace_bytes(int N, int nchi, int T, int chunk)
{
    // nine pieces, each rounded up to 256 bytes by the carving in fftlog_impl
    const FftlogLayout L = fftlog_layout(N);
    return sizeof(double2) * (8 * L.ld + 4 * (size_t)T * (L.ld + L.ldw) + (size_t)nchi * L.ldh +
                              (size_t)chunk * 3 * (L.ldt + (size_t)T * L.ld)) +
           sizeof(double) * (size_t)chunk * 3 * (nchi + (size_t)T * T) + 9 * 256;
}

z3_status fftlog_impl(int N, const double *Pk, double k_min, double k_max, const double *nu, int nchi, double chi_min,
                      double chi_max, int nmodels, const double *F, int T, const double *theta, double *out,
                      void *ws, int chunk, hipStream_t s)
{
    const FftlogLayout L = fftlog_layout(N);
    FftlogArgs g;
    g.N = N;
    g.Ns = N + 1;
    g.ld = (int)L.ld;
    g.ldw = (int)L.ldw;
    g.ldh = (int)L.ldh;
    g.Pk = Pk;
    g.k_min = k_min;
    g.k_max = k_max;
    const int ns[4] = {0, 1, 1, 2}, mts[4] = {0, 1, -1, 0};
    for (int f = 0; f < 4; ++f) g.f[f] = FactorSpec{ns[f], mts[f], nu[f]};
    g.nchi = nchi;
    g.chi_min = chi_min;
    g.dlnchi = log(chi_max / chi_min) / (nchi - 1);
    g.T = T;
    g.theta = theta;
    char *p = static_cast<char *>(ws);
    auto take = [&](size_t bytes) { char *q = p; p += (bytes + 255) / 256 * 256; return q; };
    g.cg = reinterpret_cast<double2 *>(take(4 * L.ld * sizeof(double2)));
    g.a = reinterpret_cast<double2 *>(take(4 * L.ld * sizeof(double2)));
    g.U = reinterpret_cast<double2 *>(take(4 * (size_t)T * L.ld * sizeof(double2)));
    g.Uw = reinterpret_cast<double2 *>(take(4 * (size_t)T * L.ldw * sizeof(double2)));
    g.E = reinterpret_cast<double2 *>(take((size_t)nchi * L.ldh * sizeof(double2)));
    double *D = reinterpret_cast<double *>(take((size_t)chunk * 3 * nchi * sizeof(double)));
    double2 *H = reinterpret_cast<double2 *>(take((size_t)chunk * 3 * L.ldt * sizeof(double2)));
    double2 *UA = reinterpret_cast<double2 *>(take((size_t)chunk * 3 * T * L.ld * sizeof(double2)));
    double *Ire = reinterpret_cast<double *>(take((size_t)chunk * 3 * T * T * sizeof(double)));

    hipLaunchKernelGGL(k_fftlog_coeffs, dim3((unsigned)g.Ns, 4), dim3(64), 0, s, g);
    z3_status st = check_launch("k_fftlog_coeffs");
    if (st != Z3_OK) return st;
    const int64_t nop = (int64_t)4 * T * g.Ns;
    hipLaunchKernelGGL(k_fftlog_operands, dim3((unsigned)((nop + 255) / 256)), dim3(256), 0, s, g);
    if ((st = check_launch("k_fftlog_operands")) != Z3_OK) return st;
    const int64_t nph = (int64_t)nchi * (N + 1);
    hipLaunchKernelGGL(k_fftlog_phases, dim3((unsigned)((nph + 255) / 256)), dim3(256), 0, s, g);
    if ((st = check_launch("k_fftlog_phases")) != Z3_OK) return st;
    // factor pairs of A_0, A_1, A_2: (0,0)x(0,0), (1,1)x(1,-1), (2,0)x(2,0)
    const int f1[3] = {0, 1, 3}, f2[3] = {0, 2, 3};
    const double3 nusum = make_double3(nu[0] + nu[0], nu[1] + nu[2], nu[3] + nu[3]);
    const int64_t ld = (int64_t)L.ld, ldw = (int64_t)L.ldw, ldh = (int64_t)L.ldh, ldt = (int64_t)L.ldt;
    for (int b0 = 0; b0 < nmodels && st == Z3_OK; b0 += chunk) {
        const int nb = nmodels - b0 < chunk ? nmodels - b0 : chunk;
        const int64_t nw = (int64_t)nb * nchi * 3;
        hipLaunchKernelGGL(k_fftlog_weights, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s,
                           F + (size_t)b0 * nchi, nchi, nb, chi_min, g.dlnchi, nusum, D);
        if ((st = check_launch("k_fftlog_weights")) != Z3_OK) break;
        // h[col][N + t] = sum_j E[j][t] D[col][j] for t = 0..N, mirrored to N - t; col = (q, b)
        CGemm mh{g.E, 1, ldh, 0, D, 1, (int64_t)nchi, 0, H + N, 1, ldt, 0, N + 1, 3 * nb, nchi};
        if ((st = cgemm<1, 1, true>(mh, 1, s)) != Z3_OK) break;
        for (int q = 0; q < 3 && st == Z3_OK; ++q) {
            // UA[b][q][i][s2] = sum_{m >= 0} Uw_f1[i][m] h[q][b][N/2 + m + s2]
            CGemm m2{g.Uw + (size_t)f1[q] * T * ldw, ldw, 1, 0,
                     H + (size_t)q * nb * ldt + N / 2, 1, 1, ldt,
                     UA + (size_t)q * T * ld, ld, 1, 3 * T * ld, T, g.Ns, N / 2 + 1};
            st = cgemm<2, 4, false>(m2, nb, s);
            // Ire[b][q] = Re(UA[b][q] U_f2^T)
            CGemm m3{UA + (size_t)q * T * ld, ld, 1, 3 * T * ld,
                     g.U + (size_t)f2[q] * T * ld, 1, ld, 0,
                     Ire + (size_t)q * T * T, (int64_t)T, 1, (int64_t)3 * T * T, T, T, g.Ns};
            if (st == Z3_OK) st = cgemm<3, 4, true>(m3, nb, s);
        }
        if (st != Z3_OK) break;
        const int64_t no = (int64_t)nb * 3 * T * T;
        hipLaunchKernelGGL(k_fftlog_out, dim3((unsigned)((no + 255) / 256)), dim3(256), 0, s, Ire, T, nb,
                           out + (size_t)b0 * 3 * T * T);
        st = check_launch("k_fftlog_out");
    }
    return st;
}

}  // namespace z3
