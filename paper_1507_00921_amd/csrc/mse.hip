// Loss head of the differentiation workload: the mean squared error between the
// detected symbols and the transmitted ones (Sec. IV footnote), and its reverse
// mode.  Definitions and conventions in include/dbp.h.
//
// With L samples per signal and polarization, L2 = L / 2 symbols and L4 = L / 4,
// the receive filter mf (real, on the length-L DFT grid) followed by taking the
// even samples is
//
//   y[2m] = (1/L) sum_{k<L} X[k] mf[k] e^{+2 pi i k m / L2},   X = DFT_L(z),
//
// and is evaluated without a length-L transform:
//   * splitting n = n' + L2 j gives the even and odd bins as two L2-point
//     transforms, X[2k + h] = DFT_L2(v_h)[k] with v_h[n'] = (z[n'] + (-1)^h
//     z[n' + L2]) W_L^{h n'};
//   * the folded spectrum F[k''] = X[k''] mf[k''] + X[k'' + L2] mf[k'' + L2] of the
//     decimated output splits by the parity h of k'' = 2k + h into two L4-point
//     inverse transforms A_h (each workgroup of the fold kernel owns one h);
//   * y[2m] = (A_0[m mod L4] + W_L2^{-m} A_1[m mod L4]) / L.
// The reverse mode runs the same factorisation backwards: the residual gradient
// u (one value per symbol) is zero-inserted, so DFT_L of it is DFT_L2(u)
// repeated, and the length-L inverse transform of U[k mod L2] mf[k] splits by the
// parity of k into two L2-point inverse transforms combined with W_L^{-n}.
//
// Kernels (T = L2 / 16 threads per workgroup):
//   mse_fold_kernel      grid (signals, 2): v_h, its L2-point FFT, the fold with mf,
//                        the L4-point inverse FFT -> A_h
//   mse_residual_kernel  grid signals: y, the residual a = y / amp - s, per-signal sum
//                        of |a|^2 (FP32 per thread, FP64 across the workgroup)
//   mse_sum_kernel       one workgroup: the per-signal sums added in FP64 in order
//   mse_adj_fft_kernel   grid signals: u = a * 2 g / (amp n_tot), U = DFT_L2(u)
//   mse_adj_half_kernel  grid (signals, 2): the L2-point inverse FFT of
//                        U[(2k + h) mod L2] mf[2k + h] -> R_h
//   mse_adj_combine      grad[n] = (R_0[n mod L2] + W_L^{-n} R_1[n mod L2]) / L
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "alloc.hpp"
#include "dbp.h"
#include "fft.hpp"

namespace dbp {
namespace mse {

constexpr int E2 = 16;   // values per thread of the L2-point transforms
constexpr int E4 = 8;    // values per thread of the L4-point transforms

template <int L2> struct Shape {
    static constexpr int L = 2 * L2, L4 = L2 / 2, T = L2 / E2;
    static_assert(L4 / E4 == T, "both transforms on the same threads");
    static constexpr int LDS2 = Exchange<L2, E2, 1>::FLOATS2;
    static constexpr int LDS4 = Exchange<L4, E4, 1>::FLOATS2;
    static constexpr int LDS = LDS2 > LDS4 ? LDS2 : LDS4;
};

struct Tables {
    const float2* tw2;   // exp(-2 pi i q / L2), q < L2: the L2-point transforms and W_L2^m
    const float2* tw4;   // exp(-2 pi i q / L4), q < L4
    const float2* twl;   // exp(-2 pi i q / L), q < L2: W_L^n (and -W_L^{n-L2} above)
    const float* mf;     // receive filter on the length-L grid
};

// W_L^n = exp(-2 pi i n / L) for 0 <= n < L from the half table
__device__ __forceinline__ float2 w_l(const float2* __restrict__ twl, int n, int l2) {
    const float2 w = twl[n < l2 ? n : n - l2];
    return n < l2 ? w : make_float2(-w.x, -w.y);
}

template <int L2>
__global__ __launch_bounds__(L2 / E2) void mse_fold_kernel(const float2* __restrict__ z, float2* __restrict__ ab,
                                                           Tables tb) {
    using S = Shape<L2>;
    __shared__ float2 lds[S::LDS];
    const int t = threadIdx.x, h = blockIdx.y;
    const long long sig = blockIdx.x;
    const float2* __restrict__ x = z + sig * S::L;
    float2 v[1][E2];
#pragma unroll
    for (int q = 0; q < E2; ++q) {
        const int n = t + S::T * q;
        const float2 a = x[n], b = x[n + L2];
        v[0][q] = h == 0 ? cadd(a, b) : cmul(csub(a, b), tb.twl[n]);
    }
    {
        TwReg<L2, E2> twr;
        load_twiddles<L2, E2>(twr, tb.tw2, t);
        block_fft<L2, E2, 1, false>(v, lds, twr, t);
    }
    // v[0][q] = V_h[t + T q]; F_h[k] = V_h[k] mf[2k + h] + V_h[k + L4] mf[2k + h + L2], k = t + T q
    float2 f[1][E4];
#pragma unroll
    for (int q = 0; q < E4; ++q) {
        const int k = t + S::T * q;
        const float m0 = tb.mf[2 * k + h], m1 = tb.mf[2 * k + h + L2];
        const float2 a = v[0][q], b = v[0][q + E4];
        f[0][q] = make_float2(fmaf(a.x, m0, b.x * m1), fmaf(a.y, m0, b.y * m1));
    }
    __syncthreads();   // the L2 transform's last exchange is read by every thread before LDS is reused
    {
        TwReg<S::L4, E4> twr;
        load_twiddles<S::L4, E4>(twr, tb.tw4, t);
        block_fft<S::L4, E4, 1, true>(f, lds, twr, t);
    }
    float2* __restrict__ o = ab + (sig * 2 + h) * S::L4;
#pragma unroll
    for (int q = 0; q < E4; ++q) o[t + S::T * q] = f[0][q];
}

// Sum of one value per thread over the workgroup in FP64, in a fixed order.
template <int T> __device__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = T / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    return red[0];
}

template <int L2>
__global__ __launch_bounds__(L2 / E2) void mse_residual_kernel(const float2* __restrict__ ab,
                                                               const float2* __restrict__ sym,
                                                               float2* __restrict__ res, double* __restrict__ part,
                                                               Tables tb, float inv_l_amp) {
    using S = Shape<L2>;
    __shared__ double red[S::T];
    const int t = threadIdx.x;
    const long long sig = blockIdx.x;
    const float2* __restrict__ a0 = ab + sig * 2 * S::L4;
    const float2* __restrict__ a1 = a0 + S::L4;
    const float2* __restrict__ s = sym + sig * L2;
    float2* __restrict__ r = res + sig * L2;
    float acc = 0.f;
#pragma unroll
    for (int q = 0; q < E2; ++q) {
        const int m = t + S::T * q, mm = t + S::T * (q & (E4 - 1));
        // y[2m] / amp = (A_0 + conj(W_L2^m) A_1) / (L amp)
        const float2 y = cadd(a0[mm], cmulc(a1[mm], tb.tw2[m]));
        const float2 sv = s[m];
        const float2 d = make_float2(fmaf(y.x, inv_l_amp, -sv.x), fmaf(y.y, inv_l_amp, -sv.y));
        r[m] = d;
        acc = fmaf(d.x, d.x, fmaf(d.y, d.y, acc));
    }
    const double tot = block_sum<S::T>((double)acc, red);
    if (t == 0) part[sig] = tot;
}

// One workgroup of 256 threads: thread j sums signals j, j + 256, ... in order,
// then the 256 sums are added pairwise in a fixed tree.
__global__ __launch_bounds__(256) void mse_sum_kernel(const double* __restrict__ part, int n_sig, double inv_n,
                                                      float* __restrict__ loss) {
    __shared__ double red[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < n_sig; i += 256) v += part[i];
    const double tot = block_sum<256>(v, red);
    if (threadIdx.x == 0) *loss = (float)(tot * inv_n);
}

template <int L2>
__global__ __launch_bounds__(L2 / E2) void mse_adj_fft_kernel(const float2* __restrict__ res,
                                                              const float* __restrict__ grad_loss,
                                                              float2* __restrict__ U, Tables tb, float scale) {
    using S = Shape<L2>;
    __shared__ float2 lds[S::LDS2];
    const int t = threadIdx.x;
    const long long sig = blockIdx.x;
    const float g = grad_loss ? *grad_loss * scale : scale;   // 2 dL/dloss / (amp n_tot)
    const float2* __restrict__ r = res + sig * L2;
    float2 v[1][E2];
#pragma unroll
    for (int q = 0; q < E2; ++q) {
        const float2 d = r[t + S::T * q];
        v[0][q] = make_float2(d.x * g, d.y * g);
    }
    TwReg<L2, E2> twr;
    load_twiddles<L2, E2>(twr, tb.tw2, t);
    block_fft<L2, E2, 1, false>(v, lds, twr, t);
    float2* __restrict__ o = U + sig * L2;
#pragma unroll
    for (int q = 0; q < E2; ++q) o[t + S::T * q] = v[0][q];
}

template <int L2>
__global__ __launch_bounds__(L2 / E2) void mse_adj_half_kernel(const float2* __restrict__ U,
                                                               float2* __restrict__ R, Tables tb) {
    using S = Shape<L2>;
    __shared__ float2 lds[S::LDS2];
    const int t = threadIdx.x, h = blockIdx.y;
    const long long sig = blockIdx.x;
    const float2* __restrict__ u = U + sig * L2;
    float2 v[1][E2];
#pragma unroll
    for (int q = 0; q < E2; ++q) {
        const int k = t + S::T * q;              // k' < L2; bin 2k' + h of the length-L grid
        const int b = 2 * k + h;
        const float m = tb.mf[b];
        const float2 x = u[b & (L2 - 1)];
        v[0][q] = make_float2(x.x * m, x.y * m);
    }
    TwReg<L2, E2> twr;
    load_twiddles<L2, E2>(twr, tb.tw2, t);
    block_fft<L2, E2, 1, true>(v, lds, twr, t);
    float2* __restrict__ o = R + (sig * 2 + h) * L2;
#pragma unroll
    for (int q = 0; q < E2; ++q) o[t + S::T * q] = v[0][q];
}

// grid (ceil(L / 256), signals)
__global__ __launch_bounds__(256) void mse_adj_combine(const float2* __restrict__ R, float2* __restrict__ grad,
                                                       const float2* __restrict__ twl, int l2, float inv_l) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    const long long sig = blockIdx.y;
    if (n >= 2 * l2) return;
    const int nn = n & (l2 - 1);
    const float2 r0 = R[sig * 2 * l2 + nn], r1 = R[(sig * 2 + 1) * l2 + nn];
    const float2 g = cadd(r0, cmulc(r1, w_l(twl, n, l2)));   // W_L^{-n} = conj(W_L^n)
    grad[sig * 2 * l2 + n] = make_float2(g.x * inv_l, g.y * inv_l);
}

using FoldFn = hipError_t (*)(const float2*, float2*, const Tables&, int, hipStream_t);
using ResFn = hipError_t (*)(const float2*, const float2*, float2*, double*, const Tables&, float, int, hipStream_t);
using AdjFn = hipError_t (*)(const float2*, const float*, float2*, float2*, const Tables&, float, int, hipStream_t);

template <int L2> hipError_t launch_fold(const float2* z, float2* ab, const Tables& tb, int n_sig, hipStream_t s) {
    hipLaunchKernelGGL((mse_fold_kernel<L2>), dim3(n_sig, 2), dim3(L2 / E2), 0, s, z, ab, tb);
    return hipGetLastError();
}

template <int L2>
hipError_t launch_residual(const float2* ab, const float2* sym, float2* res, double* part, const Tables& tb,
                           float inv_l_amp, int n_sig, hipStream_t s) {
    hipLaunchKernelGGL((mse_residual_kernel<L2>), dim3(n_sig), dim3(L2 / E2), 0, s, ab, sym, res, part, tb,
                       inv_l_amp);
    return hipGetLastError();
}

template <int L2>
hipError_t launch_adjoint(const float2* res, const float* grad_loss, float2* U, float2* R, const Tables& tb,
                          float scale, int n_sig, hipStream_t s) {
    hipLaunchKernelGGL((mse_adj_fft_kernel<L2>), dim3(n_sig), dim3(L2 / E2), 0, s, res, grad_loss, U, tb, scale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((mse_adj_half_kernel<L2>), dim3(n_sig, 2), dim3(L2 / E2), 0, s, U, R, tb);
    return hipGetLastError();
}

struct Variant {
    int l2;
    FoldFn fold;
    ResFn residual;
    AdjFn adjoint;
};

#define DBP_MSE_V(L2) {L2, launch_fold<L2>, launch_residual<L2>, launch_adjoint<L2>}
static const Variant kVariants[] = {DBP_MSE_V(1024), DBP_MSE_V(2048), DBP_MSE_V(4096), DBP_MSE_V(8192),
                                    DBP_MSE_V(16384)};

const Variant* find_variant(long long l2) {
    for (const Variant& v : kVariants)
        if (v.l2 == l2) return &v;
    return nullptr;
}

}  // namespace mse
}  // namespace dbp

using namespace dbp::mse;

struct dbp_mse_s {
    long long L = 0;
    int n_sig = 0;                 // batch * n_pol
    double amp = 1.0;
    const Variant* var = nullptr;
    Tables tb{};
    float2* ab = nullptr;          // [n_sig][2][L4] (forward); U [n_sig][L2] (reverse)
    float2* res = nullptr;         // [n_sig][L2] residual of the last forward
    float2* R = nullptr;           // [n_sig][2][L2]
    double* part = nullptr;        // [n_sig]
    void* mem = nullptr;
    int device = -1;
};

namespace {

bool on_device(const dbp_mse_s* m) {
    int dev = -1;
    return hipGetDevice(&dev) == hipSuccess && dev == m->device;
}

void twiddles(std::vector<float2>& tw, long long n_table, long long period) {
    tw.resize((size_t)n_table);
    for (long long q = 0; q < n_table; ++q) {
        const double a = -2.0 * M_PI * (double)q / (double)period;
        tw[(size_t)q] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
}

}  // namespace

extern "C" {

dbp_status dbp_mse_create(int64_t n_samples, int32_t n_pol, int32_t batch, const double* mf, double amplitude,
                          dbp_mse_t* out) {
    if (!out) return DBP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!mf || (n_pol != 1 && n_pol != 2) || batch < 1 || !(amplitude > 0.0) || !std::isfinite(amplitude))
        return DBP_ERR_INVALID_ARG;
    if (n_samples < 2 || (n_samples & (n_samples - 1)) || (long long)batch * n_pol > (1 << 24))
        return DBP_ERR_INVALID_ARG;
    for (int64_t k = 0; k < n_samples; ++k)
        if (!std::isfinite(mf[k])) return DBP_ERR_INVALID_ARG;
    const Variant* var = find_variant(n_samples / 2);
    if (!var) return DBP_ERR_UNSUPPORTED;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DBP_ERR_HIP;
    dbp_mse_s* m = new (std::nothrow) dbp_mse_s();
    if (!m) return DBP_ERR_OOM;
    m->device = dev;
    m->L = n_samples;
    m->n_sig = batch * n_pol;
    m->amp = amplitude;
    m->var = var;
    const long long L = n_samples, l2 = L / 2, l4 = L / 4, ns = m->n_sig;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_tw2 = al(l2 * sizeof(float2)), b_tw4 = al(l4 * sizeof(float2)), b_twl = al(l2 * sizeof(float2));
    const size_t b_mf = al(L * sizeof(float));
    const size_t b_ab = al((size_t)ns * l2 * sizeof(float2)), b_res = b_ab;
    const size_t b_R = al((size_t)ns * L * sizeof(float2)), b_part = al((size_t)ns * sizeof(double));
    const size_t bytes = b_tw2 + b_tw4 + b_twl + b_mf + b_ab + b_res + b_R + b_part;
    hipError_t e = dbp::device_alloc(&m->mem, bytes);
    if (e != hipSuccess) {
        delete m;
        return e == hipErrorOutOfMemory ? DBP_ERR_OOM : DBP_ERR_HIP;
    }
    char* p = (char*)m->mem;
    float2* tw2 = (float2*)p;
    p += b_tw2;
    float2* tw4 = (float2*)p;
    p += b_tw4;
    float2* twl = (float2*)p;
    p += b_twl;
    float* mfd = (float*)p;
    p += b_mf;
    m->ab = (float2*)p;
    p += b_ab;
    m->res = (float2*)p;
    p += b_res;
    m->R = (float2*)p;
    p += b_R;
    m->part = (double*)p;
    m->tb = Tables{tw2, tw4, twl, mfd};
    std::vector<float2> t2, t4, tl;
    twiddles(t2, l2, l2);
    twiddles(t4, l4, l4);
    twiddles(tl, l2, L);
    std::vector<float> mff((size_t)L);
    for (long long k = 0; k < L; ++k) mff[(size_t)k] = (float)mf[k];
    if (hipMemcpy(tw2, t2.data(), l2 * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(tw4, t4.data(), l4 * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(twl, tl.data(), l2 * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(mfd, mff.data(), L * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        dbp_mse_destroy(m);
        return DBP_ERR_HIP;
    }
    *out = m;
    return DBP_OK;
}

dbp_status dbp_mse_forward(dbp_mse_t m, const void* z, const void* symbols, float* loss, void* stream) {
    if (!m || !z || !symbols || !loss) return DBP_ERR_INVALID_ARG;
    if (!on_device(m)) return DBP_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const double n_tot = (double)m->n_sig * (double)(m->L / 2);
    if (m->var->fold((const float2*)z, m->ab, m->tb, m->n_sig, s) != hipSuccess) return DBP_ERR_HIP;
    if (m->var->residual(m->ab, (const float2*)symbols, m->res, m->part, m->tb,
                         (float)(1.0 / ((double)m->L * m->amp)), m->n_sig, s) != hipSuccess)
        return DBP_ERR_HIP;
    hipLaunchKernelGGL(mse_sum_kernel, dim3(1), dim3(256), 0, s, m->part, m->n_sig, 1.0 / n_tot, loss);
    return hipGetLastError() == hipSuccess ? DBP_OK : DBP_ERR_HIP;
}

dbp_status dbp_mse_backward(dbp_mse_t m, const float* grad_loss, void* grad_z, void* stream) {
    if (!m || !grad_z) return DBP_ERR_INVALID_ARG;
    if (!on_device(m)) return DBP_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const double n_tot = (double)m->n_sig * (double)(m->L / 2);
    const float scale = (float)(2.0 / (m->amp * n_tot));
    if (m->var->adjoint(m->res, grad_loss, m->ab, m->R, m->tb, scale, m->n_sig, s) != hipSuccess)
        return DBP_ERR_HIP;
    const int l2 = (int)(m->L / 2);
    hipLaunchKernelGGL(mse_adj_combine, dim3((unsigned)((m->L + 255) / 256), (unsigned)m->n_sig), dim3(256), 0, s,
                       m->R, (float2*)grad_z, m->tb.twl, l2, (float)(1.0 / (double)m->L));
    return hipGetLastError() == hipSuccess ? DBP_OK : DBP_ERR_HIP;
}

void dbp_mse_destroy(dbp_mse_t m) {
    if (!m) return;
    if (m->mem) (void)hipFree(m->mem);
    delete m;
}

}  // extern "C"
