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
// The products A = X1^T diag(d) X2 (X_{chi,s} = chi^{-a_s}, d the quadrature weights times
// F chi^{-2}), U1 A and (U1 A) U2^T are complex FP64 matrix products: one batched kernel on
// v_mfma_f64_16x16x4f64 (four real products per complex 16x16x4 step).  The coefficients,
// the Gamma ratios (complex log-Gamma: upward recurrence to Re z >= 12, then Stirling's
// series) and the operands are small elementwise kernels.
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

// log Gamma(z) for complex z away from the poles (any branch of the imaginary part: only
// exp of differences is used).  Upward recurrence log Gamma(z) = log Gamma(z + K) -
// sum_{j<K} log(z + j) until Re z >= 12, then Stirling's series with Bernoulli terms
// B_{2k} / (2k (2k-1) z^{2k-1}), k = 1..8.
__device__ double2 clgamma(double2 z)
{
    double2 shift = make_double2(0.0, 0.0);
    while (z.x < 12.0) {
        const double2 l = clog(z);
        shift.x += l.x;
        shift.y += l.y;
        z.x += 1.0;
    }
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
    int N;                    // samples of P (even); Ns = N + 1 coefficients
    int Ns, ld;               // ld: padded row length of the s dimension
    const double *Pk;
    double k_min, k_max;
    FactorSpec f[4];          // (0,0), (1,1), (1,-1), (2,0)
    int nchi;
    double chi_min, dlnchi;
    int T;
    const double *theta;
    double2 *c;               // [4][ld]
    double2 *a;               // [4][ld]
    double2 *U;               // [4][T][ld]
    double2 *X;               // [4][nchi][ld]
};

// c_s and a_s of each factor: one thread per (factor, s)
__global__ void k_fftlog_coeffs(FftlogArgs g)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x, f = blockIdx.y;
    if (s >= g.ld) return;
    double2 *c = g.c + (size_t)f * g.ld, *a = g.a + (size_t)f * g.ld;
    if (s >= g.Ns) {
        c[s] = make_double2(0.0, 0.0);
        a[s] = make_double2(0.0, 0.0);
        return;
    }
    const int N = g.N, m = s - N / 2;
    const double L = log(g.k_max / g.k_min);
    const double eta = (double)(N - 1) / N * 2.0 * kPi * m / L;
    const double nu = g.f[f].nu;
    const double dl = L / (N - 1);
    double re = 0.0, im = 0.0;
    const int mm = ((m % N) + N) % N;
    for (int l = 0; l < N; ++l) {
        const double v = g.Pk[l] * exp(-nu * dl * l);
        const int q = (int)(((int64_t)mm * l) % N);  // e^{-2 pi i m l / N} from the exact residue
        double sn, cs;
        sincospi(2.0 * q / N, &sn, &cs);
        re += v * cs;
        im -= v * sn;
    }
    const double w = (s == 0 || s == N) ? 0.5 : 1.0;
    const double2 pre = cexp(make_double2(-nu * log(g.k_min), -eta * log(g.k_min)));
    const double2 d = make_double2(w * re / N, w * im / N);
    c[s] = cmul(pre, d);
    a[s] = make_double2(1.0 + nu, eta);
}

// U[f][i][s] = c_s g(a_s) theta_i^{-(1 + a_s + mt)} and X[f][j][s] = chi_j^{-a_s}
__global__ void k_fftlog_operands(FftlogArgs g)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x, f = blockIdx.y;
    if (s >= g.ld) return;
    const int n = g.f[f].n, mt = g.f[f].mt;
    const double2 c = g.c[(size_t)f * g.ld + s], a = g.a[(size_t)f * g.ld + s];
    double2 *U = g.U + (size_t)f * g.T * g.ld;
    double2 *X = g.X + (size_t)f * g.nchi * g.ld;
    if (s >= g.Ns) {
        for (int i = 0; i < g.T; ++i) U[(size_t)i * g.ld + s] = make_double2(0.0, 0.0);
        for (int j = 0; j < g.nchi; ++j) X[(size_t)j * g.ld + s] = make_double2(0.0, 0.0);
        return;
    }
    const double2 l1 = clgamma(make_double2(0.5 * (1.0 + mt + a.x + n), 0.5 * a.y));
    const double2 l2 = clgamma(make_double2(0.5 * (1.0 - a.x - mt + n), -0.5 * a.y));
    const double ln2 = 0.69314718055994530942;
    const double2 gl = make_double2((mt + a.x - 1.0) * ln2 + l1.x - l2.x, a.y * ln2 + l1.y - l2.y);
    double2 cg = cmul(c, cexp(gl));
    cg.x /= kPi;
    cg.y /= kPi;
    for (int i = 0; i < g.T; ++i) {
        const double lt = log(g.theta[i]);
        U[(size_t)i * g.ld + s] = cmul(cg, cexp(make_double2(-(1.0 + a.x + mt) * lt, -a.y * lt)));
    }
    for (int j = 0; j < g.nchi; ++j) {
        const double lc = log(g.chi_min) + j * g.dlnchi;
        X[(size_t)j * g.ld + s] = cexp(make_double2(-a.x * lc, -a.y * lc));
    }
}

// quadrature weights of each model: d[b][j] = w_j chi_j F_b(chi_j) chi_j^{-2}
__global__ void k_fftlog_weights(const double *F, int nchi, int nmodels, double chi_min, double dlnchi, double *d)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nchi * nmodels) return;
    const int j = (int)(t % nchi);
    const double chi = exp(log(chi_min) + j * dlnchi);
    const double w = (j == 0 || j == nchi - 1) ? 0.5 * dlnchi : dlnchi;
    d[t] = w * F[t] / chi;
}

// Batched complex FP64 product C[b] = A[b] B[b] (optionally A scaled per k by dsc[b][k]),
// elements addressed by strides; one wave per 16 x 16 tile of C, 2 x 2 waves per block.
struct CGemm {
    const double2 *A;
    int64_t a_i, a_k, a_b;
    const double2 *B;
    int64_t b_k, b_j, b_b;
    double2 *C;
    int64_t c_i, c_j, c_b;
    const double *dsc;        // [batch][K] or null
    int M, N, K;
};

// SCALE: the chi-quadrature product X1^T diag(d) X2 (dsc set); its own kernel name so that
// profiles separate it from the two small products
template <bool SCALE>
__global__ __launch_bounds__(256) void k_cgemm(CGemm g)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = blockIdx.z;
    const int i0 = (blockIdx.y * 2 + (w >> 1)) * 16, j0 = (blockIdx.x * 2 + (w & 1)) * 16;
    const int r = lane & 15, q = lane >> 4;
    const int ia = i0 + r, jb = j0 + r;
    const double2 *A = g.A + (size_t)b * g.a_b;
    const double2 *B = g.B + (size_t)b * g.b_b;
    const double *dsc = SCALE ? g.dsc + (size_t)b * g.K : nullptr;
    v4d re = {0.0, 0.0, 0.0, 0.0}, im = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < g.K; k0 += 16) {
        double2 av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + 4 * u + q;
            const bool in = k < g.K;
            av[u] = (in && ia < g.M) ? A[ia * g.a_i + k * g.a_k] : make_double2(0.0, 0.0);
            bv[u] = (in && jb < g.N) ? B[k * g.b_k + jb * g.b_j] : make_double2(0.0, 0.0);
            if (SCALE && in) {
                const double d = dsc[k];
                av[u].x *= d;
                av[u].y *= d;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            re = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].x, bv[u].x, re, 0, 0, 0);
            re = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[u].y, bv[u].y, re, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].x, bv[u].y, im, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u].y, bv[u].x, im, 0, 0, 0);
        }
    }
    // v_mfma_f64_16x16x4f64 result layout: register k of lane l holds D[4k + l/16][l % 16]
    double2 *C = g.C + (size_t)b * g.c_b;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = i0 + 4 * k + q, j = j0 + r;
        if (i < g.M && j < g.N) C[i * g.c_i + j * g.c_j] = make_double2(re[k], im[k]);
    }
}

static z3_status cgemm(const CGemm &g, int batch, hipStream_t s)
{
    const dim3 grid((unsigned)((g.N + 31) / 32), (unsigned)((g.M + 31) / 32), (unsigned)batch);
    if (!g.dsc) {
        hipLaunchKernelGGL(k_cgemm<false>, grid, dim3(256), 0, s, g);
        return check_launch("k_cgemm");
    }
    hipEvent_t ev0;
    profile_begin(s, &ev0);
    hipLaunchKernelGGL(k_cgemm<true>, grid, dim3(256), 0, s, g);
    profile_end(s, ev0);
    return check_launch("k_cgemm");
}

// out[b][0] = Re I0, out[b][1] = Re (I1 + I1^T), out[b][2] = Re I2
__global__ void k_fftlog_out(const double2 *I, int T, int nmodels, double *out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)T * T;
    if (t >= per * 3 * nmodels) return;
    const int64_t b = t / (3 * per), rem = t % (3 * per);
    const int p = (int)(rem / per), ij = (int)(rem % per), i = ij / T, j = ij % T;
    const double2 *Ib = I + (size_t)(b * 3 + p) * per;
    double v = Ib[ij].x;
    if (p == 1) v += Ib[(size_t)j * T + i].x;
    out[t] = v;
}

size_t fftlog_workspace_bytes(int N, int nchi, int T, int chunk)
{
    // eight pieces, each rounded up to 256 bytes by the carving in fftlog_impl
    const size_t ld = (size_t)((N + 1 + 15) / 16 * 16);
    return sizeof(double2) * (8 * ld + 4 * (size_t)T * ld + 4 * (size_t)nchi * ld +
                              (size_t)chunk * 3 * (ld * ld + (size_t)T * ld + (size_t)T * T)) +
           sizeof(double) * (size_t)chunk * nchi + 8 * 256;
}

z3_status fftlog_impl(int N, const double *Pk, double k_min, double k_max, const double *nu, int nchi, double chi_min,
                      double chi_max, int nmodels, const double *F, int T, const double *theta, double *out,
                      void *ws, int chunk, hipStream_t s)
{
    FftlogArgs g;
    g.N = N;
    g.Ns = N + 1;
    g.ld = (N + 1 + 15) / 16 * 16;
    g.Pk = Pk;
    g.k_min = k_min;
    g.k_max = k_max;
    const int ns[4] = {0, 1, 1, 2}, mts[4] = {0, 1, -1, 0};
    for (int f = 0; f < 4; ++f) g.f[f] = FactorSpec{ns[f], mts[f], nu[f]};
    g.nchi = nchi;
    g.chi_min = chi_min;
    g.dlnchi = nchi > 1 ? log(chi_max / chi_min) / (nchi - 1) : 0.0;
    g.T = T;
    g.theta = theta;
    const size_t ld = (size_t)g.ld;
    char *p = static_cast<char *>(ws);
    auto take = [&](size_t bytes) { char *q = p; p += (bytes + 255) / 256 * 256; return q; };
    g.c = reinterpret_cast<double2 *>(take(4 * ld * sizeof(double2)));
    g.a = reinterpret_cast<double2 *>(take(4 * ld * sizeof(double2)));
    g.U = reinterpret_cast<double2 *>(take(4 * (size_t)T * ld * sizeof(double2)));
    g.X = reinterpret_cast<double2 *>(take(4 * (size_t)nchi * ld * sizeof(double2)));
    double2 *Am = reinterpret_cast<double2 *>(take((size_t)chunk * 3 * ld * ld * sizeof(double2)));
    double2 *UA = reinterpret_cast<double2 *>(take((size_t)chunk * 3 * T * ld * sizeof(double2)));
    double2 *Im = reinterpret_cast<double2 *>(take((size_t)chunk * 3 * T * T * sizeof(double2)));
    double *d = reinterpret_cast<double *>(take((size_t)chunk * nchi * sizeof(double)));

    const dim3 gs((unsigned)((ld + 63) / 64), 4);
    hipLaunchKernelGGL(k_fftlog_coeffs, gs, dim3(64), 0, s, g);
    z3_status st = check_launch("k_fftlog_coeffs");
    if (st != Z3_OK) return st;
    hipLaunchKernelGGL(k_fftlog_operands, gs, dim3(64), 0, s, g);
    if ((st = check_launch("k_fftlog_operands")) != Z3_OK) return st;
    // factor pairs of A_0, A_1, A_2: (0,0)x(0,0), (1,1)x(1,-1), (2,0)x(2,0)
    const int f1[3] = {0, 1, 3}, f2[3] = {0, 2, 3};
    for (int b0 = 0; b0 < nmodels && st == Z3_OK; b0 += chunk) {
        const int nb = nmodels - b0 < chunk ? nmodels - b0 : chunk;
        const int64_t nw = (int64_t)nb * nchi;
        hipLaunchKernelGGL(k_fftlog_weights, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s,
                           F + (size_t)b0 * nchi, nchi, nb, chi_min, g.dlnchi, d);
        if ((st = check_launch("k_fftlog_weights")) != Z3_OK) break;
        for (int q = 0; q < 3 && st == Z3_OK; ++q) {
            // A[b][q] = X_f1^T diag(d_b) X_f2
            CGemm m1{g.X + (size_t)f1[q] * nchi * ld, 1, (int64_t)ld, 0,
                     g.X + (size_t)f2[q] * nchi * ld, (int64_t)ld, 1, 0,
                     Am + (size_t)q * ld * ld, (int64_t)ld, 1, (int64_t)(3 * ld * ld), d, g.Ns, g.Ns, nchi};
            st = cgemm(m1, nb, s);
            // UA[b][q] = U_f1 A[b][q]
            CGemm m2{g.U + (size_t)f1[q] * T * ld, (int64_t)ld, 1, 0,
                     Am + (size_t)q * ld * ld, (int64_t)ld, 1, (int64_t)(3 * ld * ld),
                     UA + (size_t)q * T * ld, (int64_t)ld, 1, (int64_t)(3 * T * ld), nullptr, T, g.Ns, g.Ns};
            if (st == Z3_OK) st = cgemm(m2, nb, s);
            // I[b][q] = UA[b][q] U_f2^T
            CGemm m3{UA + (size_t)q * T * ld, (int64_t)ld, 1, (int64_t)(3 * T * ld),
                     g.U + (size_t)f2[q] * T * ld, 1, (int64_t)ld, 0,
                     Im + (size_t)q * T * T, (int64_t)T, 1, (int64_t)(3 * T * T), nullptr, T, T, g.Ns};
            if (st == Z3_OK) st = cgemm(m3, nb, s);
        }
        if (st != Z3_OK) break;
        const int64_t no = (int64_t)nb * 3 * T * T;
        hipLaunchKernelGGL(k_fftlog_out, dim3((unsigned)((no + 255) / 256)), dim3(256), 0, s, Im, T, nb,
                           out + (size_t)b0 * 3 * T * T);
        st = check_launch("k_fftlog_out");
    }
    return st;
}

}  // namespace z3
