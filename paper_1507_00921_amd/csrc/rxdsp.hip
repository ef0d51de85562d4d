// Receiver DSP after backpropagation (Sec. IV): resampling to two samples per
// symbol, a 2x2 butterfly equalizer trained by least squares, carrier-phase
// recovery and decisions.  Definitions and conventions in include/dbp.h.
//
// Kernels:
//   rs_kernel      one output sample per thread, K-tap polyphase FIR over the
//                  workgroup's input window in LDS (the table holds the windowed
//                  sinc of every output phase, made in FP64)
//   gram_kernel    per chunk of training symbols, every entry of U^H U and U^H s
//                  (FP32 sums over the chunk's regressors staged in LDS)
//   gram_reduce    the chunk sums added in FP64, chunk by chunk in order
//   solve_kernel   one workgroup: the normal equations solved in FP64 (Gaussian
//                  elimination with partial pivoting), the taps written as complex64
//   eq_kernel      one symbol (both polarizations) per thread, taps in LDS
//   cpr_theta      per 256-symbol block and polarization: fourth-power window
//                  sums from an LDS tile, the phase estimate, its wrapped
//                  differences and their prefix sum inside the block
//   cpr_offsets    the blocks' totals summed in order (FP64): block offsets
//   cpr_quadrant   the quarter turn that best aligns the known leading symbols
//   cpr_apply      derotation, decisions, per-block error counts
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "alloc.hpp"
#include "dbp.h"

namespace dbp {
namespace rxdsp {

constexpr int THREADS = 256;
constexpr int GRAM_CH = 128;       // training symbols per chunk
constexpr int CPR_B = 256;         // symbols per phase-recovery block
constexpr int MAX_TAPS_RS = 64;
constexpr int MAX_TAPS_EQ = 31;
constexpr int MAX_HALF_WINDOW = 256;

__device__ __forceinline__ long long wrap_index(long long i, long long n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// grid (ceil(n_out / 256), 2): 256 consecutive outputs of one polarization; their input
// window (at most 256 down / up + K + 1 samples, down <= up) is staged in LDS once.
__global__ __launch_bounds__(THREADS) void rs_kernel(const float2* __restrict__ in, float2* __restrict__ out,
                                                     long long n_in, long long n_out, int up, int down, int K,
                                                     const float* __restrict__ table) {
    extern __shared__ float2 xs[];
    const int p = blockIdx.y, t = threadIdx.x;
    const long long m0 = (long long)blockIdx.x * THREADS;
    const long long m_last = (m0 + THREADS < n_out ? m0 + THREADS : n_out) - 1;
    const long long i0 = (m0 * down) / up - K / 2 + 1;
    const int span = (int)((m_last * down) / up - K / 2 + 1 + K - i0);
    const float2* __restrict__ x = in + p * n_in;
    for (int e = t; e < span; e += THREADS) {
        long long j = i0 + e;                  // within (-K, n_in + K): n_in >= K
        j = j < 0 ? j + n_in : (j >= n_in ? j - n_in : j);
        xs[e] = x[j];
    }
    __syncthreads();
    const long long m = m0 + t;
    if (m > m_last) return;
    const long long md = m * down;
    const long long base = md / up;
    const int ph = (int)(md - base * up);
    const float* __restrict__ h = table + (long long)ph * K;
    const float2* xw = xs + (base - K / 2 + 1 - i0);
    float ax = 0.f, ay = 0.f;
#pragma unroll 8
    for (int k = 0; k < K; ++k) {
        const float2 v = xw[k];
        const float w = h[k];
        ax = fmaf(w, v.x, ax);
        ay = fmaf(w, v.y, ay);
    }
    out[p * n_out + m] = make_float2(ax, ay);
}

// Regressor element i < 2N of symbol k: x_q[(2k + j - N/2) mod n2], q = i / N, j = i % N.
// Entry e < 4N^2: R[e / 2N][e % 2N] = sum_k conj(u_k[i]) u_k[l]; then P[i][p] = sum_k conj(u_k[i]) s_p[k].
__global__ __launch_bounds__(THREADS) void gram_kernel(const float2* __restrict__ x2, long long n2,
                                                       const float2* __restrict__ sym, long long n_sym,
                                                       long long n_train, int N, float2* __restrict__ part) {
    extern __shared__ float2 sm[];
    const int TL = 2 * GRAM_CH + N;            // staged positions per polarization
    float2* tile = sm;                         // [2][TL]
    float2* st = sm + 2 * TL;                  // [2][GRAM_CH]
    const long long k0 = (long long)blockIdx.x * GRAM_CH;
    const int nk = (int)(k0 + GRAM_CH <= n_train ? GRAM_CH : n_train - k0);
    const int c = N / 2;
    for (int e = threadIdx.x; e < 2 * TL; e += THREADS) {
        const int q = e / TL, o = e - q * TL;
        tile[e] = x2[q * n2 + wrap_index(2 * k0 - c + o, n2)];
    }
    for (int e = threadIdx.x; e < 2 * GRAM_CH; e += THREADS) {
        const int p = e / GRAM_CH, o = e - p * GRAM_CH;
        st[e] = o < nk ? sym[p * n_sym + k0 + o] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const int M = 2 * N;
    const int E = M * M + 2 * M;
    float2* __restrict__ out = part + (long long)blockIdx.x * E;
    for (int e = threadIdx.x; e < E; e += THREADS) {
        int i, l = 0, p = 0;
        const bool rhs = e >= M * M;
        if (!rhs) {
            i = e / M;
            l = e - i * M;
        } else {
            i = (e - M * M) >> 1;
            p = (e - M * M) & 1;
        }
        const float2* ui = tile + (i / N) * TL + (i % N);
        const float2* ul = tile + (l / N) * TL + (l % N);
        float ax = 0.f, ay = 0.f;
        for (int k = 0; k < nk; ++k) {
            const float2 a = ui[2 * k];
            const float2 b = rhs ? st[p * GRAM_CH + k] : ul[2 * k];
            // conj(a) b
            ax = fmaf(a.x, b.x, fmaf(a.y, b.y, ax));
            ay = fmaf(a.x, b.y, fmaf(-a.y, b.x, ay));
        }
        out[e] = make_float2(ax, ay);
    }
}

constexpr int MAX_M = 2 * MAX_TAPS_EQ;   // unknowns of the least-squares butterfly

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// Value of lane `lane` (uniform) of a wave-wide double.
__device__ __forceinline__ double lane_value(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// A x = B for the M x M normal matrix and its two right-hand sides (sum = [A row-major |
// B row-major M x 2], FP64), in the order of the textbook algorithm: for every column the
// row with the largest |a| at or below the diagonal (the first on ties) is swapped up and
// eliminated from the rows below, then back substitution.  taps[p M + i] = x[i][p].  A
// zero pivot sets *flag to 1 and writes NaN taps.
//
// Per column three phases between barriers: wave 0 finds the pivot row (a wave-wide
// reduction, one lane per row) and its reciprocal; the pivot row and the current row are
// copied aside and the factors f[i] = a[i][col] / pivot formed (the pivot row's swap taken
// into account); then every row below is updated, lane = column and wave = row modulo 4.
// The row swap is carried out by these updates (the current row takes the pivot row, the
// pivot row the current row minus its multiple), so no phase reads what another writes.
// Back substitution runs in wave 0 alone, lane = row, both right-hand sides at once: the
// unknowns are found from the last row up and each is subtracted from the rows above it.
__global__ __launch_bounds__(THREADS) void solve_kernel(const double2* __restrict__ sum, int M,
                                                        float2* __restrict__ taps, int* __restrict__ flag) {
    __shared__ double2 a[MAX_M][MAX_M + 2];
    __shared__ double2 f[MAX_M];
    __shared__ double2 prow[MAX_M + 2], crow[MAX_M + 2];
    __shared__ double2 inv_s;
    __shared__ int piv;
    __shared__ int bad;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int W = M + 2;
    for (int e = t; e < M * W; e += THREADS) {
        const int i = e / W, j = e - i * W;
        a[i][j] = j < M ? sum[i * M + j] : sum[M * M + i * 2 + (j - M)];
    }
    if (t == 0) bad = 0;
    __syncthreads();
    for (int col = 0; col < M; ++col) {
        if (wv == 0) {
            const int i = col + lane;
            double v = -1.0;
            if (i < M) v = a[i][col].x * a[i][col].x + a[i][col].y * a[i][col].y;
            int idx = i;
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(v, off);
                const int oi = __shfl_xor(idx, off);
                if (ov > v || (ov == v && oi < idx)) {
                    v = ov;
                    idx = oi;
                }
            }
            if (lane == 0) {
                piv = idx;
                if (!(v > 0.0)) bad = 1;
                else inv_s = zdiv(make_double2(1.0, 0.0), a[idx][col]);
            }
        }
        __syncthreads();
        if (bad) break;
        const int pr = piv;
        if (t < W) {
            if (t >= col) {
                prow[t] = a[pr][t];
                crow[t] = a[col][t];
            }
        } else if (t >= 64 && t - 64 < M) {
            const int i = t - 64;
            if (i > col) f[i] = zmul(i == pr ? a[col][col] : a[i][col], inv_s);
        }
        __syncthreads();
        const int j = lane;
        if (j < W && j >= col) {
            const double2 pj = prow[j];
            if (wv == 0) a[col][j] = pj;
            if (j > col) {
                for (int i = col + 1 + wv; i < M; i += 4) {
                    const double2 src = i == pr ? crow[j] : a[i][j];
                    const double2 m = zmul(f[i], pj);
                    a[i][j] = make_double2(src.x - m.x, src.y - m.y);
                }
            }
        }
        __syncthreads();
    }
    if (bad) {
        for (int e = t; e < 2 * M; e += THREADS) taps[e] = make_float2(__builtin_nanf(""), __builtin_nanf(""));
        if (t == 0) *flag = 1;
        return;
    }
    if (wv != 0) return;
    const int i = lane;
    double2 b0 = make_double2(0.0, 0.0), b1 = b0, d = b0;
    if (i < M) {
        b0 = a[i][M];
        b1 = a[i][M + 1];
        d = zdiv(make_double2(1.0, 0.0), a[i][i]);
    }
    double2 x0 = make_double2(0.0, 0.0), x1 = x0;
    for (int r = M - 1; r >= 0; --r) {
        const double2 dr = make_double2(lane_value(d.x, r), lane_value(d.y, r));
        const double2 u0 = zmul(make_double2(lane_value(b0.x, r), lane_value(b0.y, r)), dr);
        const double2 u1 = zmul(make_double2(lane_value(b1.x, r), lane_value(b1.y, r)), dr);
        if (i == r) {
            x0 = u0;
            x1 = u1;
        } else if (i < r) {
            const double2 air = a[i][r];
            const double2 m0 = zmul(air, u0), m1 = zmul(air, u1);
            b0 = make_double2(b0.x - m0.x, b0.y - m0.y);
            b1 = make_double2(b1.x - m1.x, b1.y - m1.y);
        }
    }
    if (i < M) {
        taps[i] = make_float2((float)x0.x, (float)x0.y);
        taps[M + i] = make_float2((float)x1.x, (float)x1.y);
        if (i == 0) *flag = 0;
    }
}

__global__ __launch_bounds__(THREADS) void gram_reduce(const float2* __restrict__ part, int n_chunks, int E,
                                                       double2* __restrict__ sum) {
    const int e = blockIdx.x * THREADS + threadIdx.x;
    if (e >= E) return;
    double sx = 0.0, sy = 0.0;
    for (int b = 0; b < n_chunks; ++b) {
        const float2 v = part[(long long)b * E + e];
        sx += (double)v.x;
        sy += (double)v.y;
    }
    sum[e] = make_double2(sx, sy);
}

__global__ __launch_bounds__(THREADS) void eq_kernel(const float2* __restrict__ x2, long long n2,
                                                     const float2* __restrict__ taps, int N,
                                                     float2* __restrict__ y, long long n_sym) {
    __shared__ float2 w[4 * MAX_TAPS_EQ];
    for (int e = threadIdx.x; e < 4 * N; e += THREADS) w[e] = taps[e];
    __syncthreads();
    const long long k = (long long)blockIdx.x * THREADS + threadIdx.x;
    if (k >= n_sym) return;
    const int c = N / 2;
    const bool inner = 2 * k - c >= 0 && 2 * k - c + N <= n2;
    float a0x = 0.f, a0y = 0.f, a1x = 0.f, a1y = 0.f;
    for (int q = 0; q < 2; ++q) {
        const float2* __restrict__ xq = x2 + q * n2;
        for (int j = 0; j < N; ++j) {
            const float2 v = xq[inner ? 2 * k + j - c : wrap_index(2 * k + j - c, n2)];
            const float2 w0 = w[(0 * 2 + q) * N + j], w1 = w[(1 * 2 + q) * N + j];
            a0x = fmaf(w0.x, v.x, fmaf(-w0.y, v.y, a0x));
            a0y = fmaf(w0.x, v.y, fmaf(w0.y, v.x, a0y));
            a1x = fmaf(w1.x, v.x, fmaf(-w1.y, v.y, a1x));
            a1y = fmaf(w1.x, v.y, fmaf(w1.y, v.x, a1y));
        }
    }
    y[k] = make_float2(a0x, a0y);
    y[n_sym + k] = make_float2(a1x, a1y);
}

__device__ __forceinline__ float wrap_quarter(float a) {
    constexpr float Q = 1.57079632679489661923f;
    return a - Q * rintf(a * (1.0f / Q));
}

__device__ __forceinline__ float2 fourth(float2 v) {
    const float2 s = make_float2(v.x * v.x - v.y * v.y, 2.f * v.x * v.y);
    return make_float2(s.x * s.x - s.y * s.y, 2.f * s.x * s.y);
}

// grid (n_blocks, 2): block b of polarization p covers symbols [b B, b B + B).  theta0[p]:
// the estimate at symbol 0; pre[p][k]: sum of the wrapped differences d_j over the block
// up to k (d_0 = 0); tot[p][b]: the block's total.
__global__ __launch_bounds__(CPR_B) void cpr_theta(const float2* __restrict__ y, long long n_sym, int W,
                                                   float* __restrict__ theta0, float* __restrict__ pre,
                                                   float* __restrict__ tot, int n_blocks) {
    __shared__ float2 y4[CPR_B + 1 + 2 * MAX_HALF_WINDOW];
    __shared__ float th[CPR_B + 1];
    __shared__ float sc[CPR_B];
    const int p = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
    const long long k0 = (long long)b * CPR_B;
    const float2* __restrict__ yp = y + p * n_sym;
    const int TL = CPR_B + 1 + 2 * W;          // symbols k0 - 1 - W .. k0 + B + W - 1
    for (int e = t; e < TL; e += CPR_B) y4[e] = fourth(yp[wrap_index(k0 - 1 - W + e, n_sym)]);
    __syncthreads();
    // theta at k0 - 1 + s for s = 0 .. B (position s of th)
    for (int s = t; s <= CPR_B; s += CPR_B) {
        float ax = 0.f, ay = 0.f;
        for (int j = 0; j <= 2 * W; ++j) {
            ax += y4[s + j].x;
            ay += y4[s + j].y;
        }
        th[s] = atan2f(-ay, -ax) * 0.25f;
    }
    __syncthreads();
    const long long k = k0 + t;
    const bool in = k < n_sym;
    float d = (in && k > 0) ? wrap_quarter(th[t + 1] - th[t]) : 0.f;
    if (b == 0 && t == 0) theta0[p] = th[1];
    // inclusive prefix over the block (Hillis-Steele, fixed order)
    sc[t] = d;
    __syncthreads();
    for (int off = 1; off < CPR_B; off <<= 1) {
        const float v = t >= off ? sc[t - off] : 0.f;
        __syncthreads();
        sc[t] += v;
        __syncthreads();
    }
    if (in) pre[p * n_sym + k] = sc[t];
    if (t == CPR_B - 1) tot[p * n_blocks + b] = sc[t];
}

// Exclusive prefix of the block totals in FP64, one workgroup per polarization: thread t
// sums its contiguous segment of blocks, thread 0 scans the segment sums in order, then each
// thread writes its segment's offsets (a fixed order of additions for a given n_blocks).
__global__ __launch_bounds__(THREADS) void cpr_offsets(const float* __restrict__ tot, int n_blocks,
                                                       double* __restrict__ offs) {
    __shared__ double seg[THREADS];
    const int p = blockIdx.x, t = threadIdx.x;
    const int per = (n_blocks + THREADS - 1) / THREADS;
    const int b0 = t * per, b1 = min(n_blocks, b0 + per);
    const float* __restrict__ tp = tot + (long long)p * n_blocks;
    double s = 0.0;
    for (int b = b0; b < b1; ++b) s += (double)tp[b];
    seg[t] = s;
    __syncthreads();
    if (t == 0) {
        double run = 0.0;
        for (int i = 0; i < THREADS; ++i) {
            const double v = seg[i];
            seg[i] = run;
            run += v;
        }
    }
    __syncthreads();
    double run = seg[t];
    double* __restrict__ op = offs + (long long)p * n_blocks;
    for (int b = b0; b < b1; ++b) {
        op[b] = run;
        run += (double)tp[b];
    }
}

// Quarter-turn ambiguity against the first n_ref known symbols: the rotation q pi/2 with q
// the nearest integer to arg(sum z_k conj(s_k)) / (pi/2), z the derotated symbols (FP64 sums,
// fixed order); 0 when n_ref = 0.  One workgroup per polarization.
constexpr int QUAD_THREADS = 1024;

__global__ __launch_bounds__(QUAD_THREADS) void cpr_quadrant(const float2* __restrict__ y, const float2* __restrict__ sym,
                                                      long long n_sym, long long n_ref,
                                                      const float* __restrict__ theta0, const float* __restrict__ pre,
                                                      const double* __restrict__ offs, int n_blocks,
                                                      float* __restrict__ qrot) {
    __shared__ double rx[QUAD_THREADS], ry[QUAD_THREADS];
    const int p = blockIdx.x, t = threadIdx.x;
    double ax = 0.0, ay = 0.0;
    for (long long k = t; k < n_ref; k += QUAD_THREADS) {
        const float phi = (float)((double)theta0[p] + offs[p * n_blocks + k / CPR_B] + (double)pre[p * n_sym + k]);
        float sn, cs;
        sincosf(phi, &sn, &cs);
        const float2 v = y[p * n_sym + k];
        const float zx = fmaf(v.x, cs, v.y * sn), zy = fmaf(v.y, cs, -v.x * sn);
        const float2 sv = sym[p * n_sym + k];
        ax += (double)zx * sv.x + (double)zy * sv.y;
        ay += (double)zy * sv.x - (double)zx * sv.y;
    }
    rx[t] = ax;
    ry[t] = ay;
    __syncthreads();
    for (int off = QUAD_THREADS / 2; off > 0; off >>= 1) {
        if (t < off) {
            rx[t] += rx[t + off];
            ry[t] += ry[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        constexpr double Q = 1.57079632679489661923;
        qrot[p] = n_ref > 0 ? (float)(Q * rint(atan2(ry[0], rx[0]) / Q)) : 0.f;
    }
}

__global__ __launch_bounds__(CPR_B) void cpr_apply(const float2* __restrict__ y, const float2* __restrict__ sym,
                                                   long long n_sym, const float* __restrict__ theta0,
                                                   const float* __restrict__ pre, const double* __restrict__ offs,
                                                   const float* __restrict__ qrot, int n_blocks,
                                                   float2* __restrict__ z, int* __restrict__ errs) {
    __shared__ int red[CPR_B];
    const int p = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
    const long long k = (long long)b * CPR_B + t;
    int e = 0;
    if (k < n_sym) {
        const float phi = (float)((double)theta0[p] + offs[p * n_blocks + b] + (double)pre[p * n_sym + k] +
                                  (double)qrot[p]);
        float sn, cs;
        sincosf(phi, &sn, &cs);
        const float2 v = y[p * n_sym + k];
        const float2 r = make_float2(fmaf(v.x, cs, v.y * sn), fmaf(v.y, cs, -v.x * sn));   // v e^{-j phi}
        z[p * n_sym + k] = r;
        if (sym) {
            const float2 s = sym[p * n_sym + k];
            e = ((r.x < 0.f) != (s.x < 0.f) ? 1 : 0) + ((r.y < 0.f) != (s.y < 0.f) ? 1 : 0);
        }
    }
    red[t] = e;
    __syncthreads();
    for (int off = CPR_B / 2; off > 0; off >>= 1) {
        if (t < off) red[t] += red[t + off];
        __syncthreads();
    }
    if (t == 0) errs[p * n_blocks + b] = red[0];
}

}  // namespace rxdsp
}  // namespace dbp

using namespace dbp::rxdsp;

struct dbp_dsp_s {
    dbp_dsp_desc d{};
    long long n_in = 0, n_out = 0, n_sym = 0;
    int n_blocks = 0;
    float* table = nullptr;        // [up][K]
    float* theta0 = nullptr;       // [2]
    float* qrot = nullptr;         // [2]
    float* pre = nullptr;          // [2][n_sym]
    float* tot = nullptr;          // [2][n_blocks]
    double* offs = nullptr;        // [2][n_blocks]
    int* errs = nullptr;           // [2][n_blocks]
    float2* gpart = nullptr;       // normal-equation chunk sums [ceil(n_sym / GRAM_CH)][E]
    double2* gsum = nullptr;       // their FP64 totals [E]
    int* flag = nullptr;           // bit 0: the last training system was singular
    void* mem = nullptr;
    int device = -1;               // the device current at create, which owns mem
};

namespace {

double kaiser_sinc(double tau, int k_half, double beta) {
    if (std::fabs(tau) >= k_half) return 0.0;
    const double r = tau / k_half;
    const double w = std::cyl_bessel_i(0.0, beta * std::sqrt(std::max(0.0, 1.0 - r * r))) / std::cyl_bessel_i(0.0, beta);
    const double s = tau == 0.0 ? 1.0 : std::sin(M_PI * tau) / (M_PI * tau);
    return s * w;
}

bool valid(const dbp_dsp_desc* d, long long n_in) {
    if (!d || n_in <= 0) return false;
    if (d->down < 1 || d->up < d->down || d->up > 4096) return false;
    if (d->resample_taps < 2 || d->resample_taps > MAX_TAPS_RS || (d->resample_taps & 1)) return false;
    if (!(d->kaiser_beta >= 0.0) || !std::isfinite(d->kaiser_beta)) return false;
    if (d->eq_taps < 1 || d->eq_taps > MAX_TAPS_EQ || !(d->eq_taps & 1)) return false;
    if (d->cpr_half_window < 0 || d->cpr_half_window > MAX_HALF_WINDOW) return false;
    if ((n_in * d->up) % d->down != 0) return false;
    const long long n_out = n_in * d->up / d->down;
    if (n_out & 1) return false;
    if (n_in < d->resample_taps || n_out / 2 < 2LL * d->cpr_half_window + 2 || n_out < 2LL * d->eq_taps) return false;
    return true;
}

int grid_of(long long n, int per) { return (int)((n + per - 1) / per); }

// The handle's memory belongs to the device current at create; calls need it current.
bool on_device(const dbp_dsp_s* s) {
    int dev = -1;
    return hipGetDevice(&dev) == hipSuccess && dev == s->device;
}

}  // namespace

extern "C" {

dbp_status dbp_dsp_create(const dbp_dsp_desc* desc, int64_t n_in, dbp_dsp_t* out) {
    if (!out) return DBP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!valid(desc, n_in)) return DBP_ERR_INVALID_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return DBP_ERR_HIP;
    dbp_dsp_s* s = new (std::nothrow) dbp_dsp_s();
    if (!s) return DBP_ERR_OOM;
    s->device = dev;
    s->d = *desc;
    s->n_in = n_in;
    s->n_out = n_in * desc->up / desc->down;
    s->n_sym = s->n_out / 2;
    s->n_blocks = grid_of(s->n_sym, CPR_B);
    const int K = desc->resample_taps, up = desc->up;
    const size_t table_b = (size_t)up * K * sizeof(float);
    const size_t nb = (size_t)s->n_blocks;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const int M = 2 * desc->eq_taps, E = M * M + 2 * M;
    const size_t gpart_b = (size_t)grid_of(s->n_sym, GRAM_CH) * E * sizeof(float2);
    const size_t bytes = al(table_b) + 2 * al(2 * sizeof(float)) + al(2 * s->n_sym * sizeof(float)) +
                         al(2 * nb * sizeof(float)) + al(2 * nb * sizeof(double)) + al(2 * nb * sizeof(int)) +
                         al(gpart_b) + al((size_t)E * sizeof(double2)) + al(sizeof(int));
    if (dbp::device_alloc(&s->mem, bytes) != hipSuccess) {
        delete s;
        return DBP_ERR_OOM;
    }
    char* m = (char*)s->mem;
    s->table = (float*)m;
    m += al(table_b);
    s->theta0 = (float*)m;
    m += al(2 * sizeof(float));
    s->qrot = (float*)m;
    m += al(2 * sizeof(float));
    s->pre = (float*)m;
    m += al(2 * s->n_sym * sizeof(float));
    s->tot = (float*)m;
    m += al(2 * nb * sizeof(float));
    s->offs = (double*)m;
    m += al(2 * nb * sizeof(double));
    s->errs = (int*)m;
    m += al(2 * nb * sizeof(int));
    s->gpart = (float2*)m;
    m += al(gpart_b);
    s->gsum = (double2*)m;
    m += al((size_t)E * sizeof(double2));
    s->flag = (int*)m;
    // windowed sinc of every output phase ph / up, taps k = -K/2 + 1 .. K/2
    std::vector<float> tab((size_t)up * K);
    for (int ph = 0; ph < up; ++ph)
        for (int k = 0; k < K; ++k)
            tab[(size_t)ph * K + k] = (float)kaiser_sinc((double)ph / up - (k - K / 2 + 1), K / 2, desc->kaiser_beta);
    if (hipMemcpy(s->table, tab.data(), table_b, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(s->flag, 0, sizeof(int)) != hipSuccess) {
        dbp_dsp_destroy(s);
        return DBP_ERR_HIP;
    }
    *out = s;
    return DBP_OK;
}

dbp_status dbp_dsp_info(dbp_dsp_t s, int64_t* n_out, int64_t* n_sym) {
    if (!s) return DBP_ERR_INVALID_ARG;
    if (n_out) *n_out = s->n_out;
    if (n_sym) *n_sym = s->n_sym;
    return DBP_OK;
}

dbp_status dbp_dsp_resample(dbp_dsp_t s, const void* in, void* out, void* stream) {
    if (!s || !in || !out) return DBP_ERR_INVALID_ARG;
    if (!on_device(s)) return DBP_ERR_INVALID_ARG;
    const char* a = (const char*)in;
    const char* b = (const char*)out;
    if (a < b + 2 * s->n_out * sizeof(float2) && b < a + 2 * s->n_in * sizeof(float2)) return DBP_ERR_INVALID_ARG;
    const size_t smem = (size_t)(THREADS + s->d.resample_taps + 2) * sizeof(float2);
    hipLaunchKernelGGL(rs_kernel, dim3(grid_of(s->n_out, THREADS), 2), dim3(THREADS), smem, (hipStream_t)stream,
                       (const float2*)in, (float2*)out, (long long)s->n_in, (long long)s->n_out, s->d.up, s->d.down,
                       s->d.resample_taps, (const float*)s->table);
    return hipGetLastError() == hipSuccess ? DBP_OK : DBP_ERR_HIP;
}

dbp_status dbp_dsp_train(dbp_dsp_t s, const void* x2, const void* sym, int64_t n_train, void* taps, void* stream) {
    if (!s || !x2 || !sym || !taps || n_train < 1 || n_train > s->n_sym) return DBP_ERR_INVALID_ARG;
    if (!on_device(s)) return DBP_ERR_INVALID_ARG;
    const int N = s->d.eq_taps, M = 2 * N, E = M * M + 2 * M;
    const int n_chunks = grid_of(n_train, GRAM_CH);
    hipStream_t st = (hipStream_t)stream;
    float2* part = s->gpart;
    double2* sum = s->gsum;
    const size_t smem = (size_t)(2 * (2 * GRAM_CH + N) + 2 * GRAM_CH) * sizeof(float2);
    hipLaunchKernelGGL(gram_kernel, dim3(n_chunks), dim3(THREADS), smem, st, (const float2*)x2, (long long)s->n_out,
                       (const float2*)sym, (long long)s->n_sym, (long long)n_train, N, part);
    hipLaunchKernelGGL(gram_reduce, dim3(grid_of(E, THREADS)), dim3(THREADS), 0, st, (const float2*)part, n_chunks, E,
                       sum);
    // W[p][q][j] = w_p[q N + j]: solve_kernel writes taps[p M + i] = x_p[i]
    hipLaunchKernelGGL(solve_kernel, dim3(1), dim3(THREADS), 0, st, (const double2*)sum, M, (float2*)taps, s->flag);
    return hipGetLastError() == hipSuccess ? DBP_OK : DBP_ERR_HIP;
}

dbp_status dbp_dsp_status(dbp_dsp_t s, int32_t* flags) {
    if (!s || !flags) return DBP_ERR_INVALID_ARG;
    if (!on_device(s)) return DBP_ERR_INVALID_ARG;
    int v = 0;
    if (hipMemcpy(&v, s->flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return DBP_ERR_HIP;
    *flags = v;
    return DBP_OK;
}

dbp_status dbp_dsp_equalize(dbp_dsp_t s, const void* x2, const void* taps, void* y, void* stream) {
    if (!s || !x2 || !taps || !y) return DBP_ERR_INVALID_ARG;
    if (!on_device(s)) return DBP_ERR_INVALID_ARG;
    const char* a = (const char*)x2;
    const char* b = (const char*)y;
    if (a < b + 2 * s->n_sym * sizeof(float2) && b < a + 2 * s->n_out * sizeof(float2)) return DBP_ERR_INVALID_ARG;
    hipLaunchKernelGGL(eq_kernel, dim3(grid_of(s->n_sym, THREADS)), dim3(THREADS), 0, (hipStream_t)stream,
                       (const float2*)x2, (long long)s->n_out, (const float2*)taps, s->d.eq_taps, (float2*)y,
                       (long long)s->n_sym);
    return hipGetLastError() == hipSuccess ? DBP_OK : DBP_ERR_HIP;
}

dbp_status dbp_dsp_cpr(dbp_dsp_t s, const void* y, const void* sym, int64_t n_ref, void* z, int64_t* bit_errors,
                       void* stream) {
    if (!s || !y || !z || n_ref < 0 || n_ref > s->n_sym || (n_ref > 0 && !sym)) return DBP_ERR_INVALID_ARG;
    if (!on_device(s)) return DBP_ERR_INVALID_ARG;
    const char* a = (const char*)y;
    const char* b = (const char*)z;
    const size_t bytes = 2 * s->n_sym * sizeof(float2);
    if (a < b + bytes && b < a + bytes) return DBP_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid(s->n_blocks, 2);
    hipLaunchKernelGGL(cpr_theta, grid, dim3(CPR_B), 0, st, (const float2*)y, (long long)s->n_sym,
                       s->d.cpr_half_window, s->theta0, s->pre, s->tot, s->n_blocks);
    hipLaunchKernelGGL(cpr_offsets, dim3(2), dim3(THREADS), 0, st, (const float*)s->tot, s->n_blocks, s->offs);
    hipLaunchKernelGGL(cpr_quadrant, dim3(2), dim3(QUAD_THREADS), 0, st, (const float2*)y, (const float2*)sym,
                       (long long)s->n_sym, (long long)n_ref, (const float*)s->theta0, (const float*)s->pre,
                       (const double*)s->offs, s->n_blocks, s->qrot);
    hipLaunchKernelGGL(cpr_apply, grid, dim3(CPR_B), 0, st, (const float2*)y, (const float2*)sym, (long long)s->n_sym,
                       (const float*)s->theta0, (const float*)s->pre, (const double*)s->offs, (const float*)s->qrot,
                       s->n_blocks, (float2*)z, s->errs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return DBP_ERR_HIP;
    if (sym && bit_errors) {
        std::vector<int> h((size_t)2 * s->n_blocks);
        e = hipMemcpyAsync(h.data(), s->errs, h.size() * sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return DBP_ERR_HIP;
        long long tot = 0;
        for (int v : h) tot += v;
        *bit_errors = tot;
    }
    return DBP_OK;
}

void dbp_dsp_destroy(dbp_dsp_t s) {
    if (!s) return;
    if (s->mem) (void)hipFree(s->mem);
    delete s;
}

}  // extern "C"
