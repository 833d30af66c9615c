// rr_prepare: whitening of the covariates in FP64 on the device.
//
// Section 2.2 assumes covariates whitened so that Sigma_X = I, and the Appendix A remark
// maps a general Sigma_X to that case through X~ = X Sigma_X^-1/2, so that
// M = Delta^T Sigma_X^-1 Delta = ||Delta~||^2.  Here Sigma_X is the sample covariance S over
// all n units (denominator n - 1) plus a ridge lambda I, lambda = ridge_rel tr(S) / d; the
// square root is its Cholesky factor L (S_lam = L L^T), and X~ = (X - 1 mu^T) L^-T.
//
// Steps (all FP64): column means; centring; S = Xc^T Xc / (n-1) (tiled GEMM); ridge;
// blocked right-looking Cholesky (diagonal block in LDS, row solves for the panel, GEMM
// update of the trailing matrix); X~ by blocked forward substitution; BF16 hi/lo and FP32
// operand records for the W X~ contraction; column sums of |X~| for the error bound.
#include <algorithm>
#include <tuple>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "rr_internal.h"

namespace rr {

constexpr int kNB = 32;   // Cholesky / solve block

// Per-column reductions over the n units: one workgroup of kRowW waves per kColW columns, wave
// w summing units w, w + kRowW, ... of its lane's column; the kRowW partial results are then
// added in wave order, so every sum has one fixed order.
constexpr int kColW = 64, kRowW = 16;

template <int K>
__device__ __forceinline__ void combine_rows(double (*part)[kRowW][kColW], const double (&v)[K], double (&out)[K]) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < K; ++q) part[q][w][l] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < K; ++q) {
        double t = 0.0;
        for (int r = 0; r < kRowW; ++r) t += part[q][r][l];
        out[q] = t;
    }
}

// Column means mu and the centred copy Xc = X - 1 mu^T (FP64), X of either precision.
__global__ __launch_bounds__(kColW * kRowW) void mean_center_kernel(const void* X, int fp32, int64_t n, int64_t d,
                                                                     int64_t ldx, double* mu, double* Xc) {
    __shared__ double part[1][kRowW][kColW];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * kColW + l;
    auto x = [&](int64_t i) {
        return fp32 ? (double)((const float*)X)[i * ldx + j] : ((const double*)X)[i * ldx + j];
    };
    double v[1] = {0.0}, t[1];
    if (j < d)
        for (int64_t i = w; i < n; i += kRowW) v[0] += x(i);
    combine_rows<1>(part, v, t);
    const double m = t[0] / (double)n;
    if (j < d) {
        if (w == 0) mu[j] = m;
        for (int64_t i = w; i < n; i += kRowW) Xc[i * d + j] = x(i) - m;
    }
}

// C[m, c] = beta * C[m, c] + alpha * sum_k A(m, k) B(c, k), A(m,k) = A[m*sam + k*sak],
// B(c,k) = B[c*sbn + k*sbk], C row-major with leading dimension ldc.  64x64 tiles.
__global__ __launch_bounds__(256) void dgemm_nt_kernel(int64_t M, int64_t N, int64_t K, double alpha,
                                                       const double* A, int64_t sam, int64_t sak,
                                                       const double* B, int64_t sbn, int64_t sbk,
                                                       double beta, double* C, int64_t ldc) {
    __shared__ double As[16][65];
    __shared__ double Bs[16][65];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t m0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    double acc[4][4] = {};
    for (int64_t k0 = 0; k0 < K; k0 += 16) {
        for (int e = threadIdx.x; e < 16 * 64; e += 256) {
            const int kk = e & 15, r = e >> 4;
            const int64_t k = k0 + kk;
            As[kk][r] = (m0 + r < M && k < K) ? A[(m0 + r) * sam + k * sak] : 0.0;
            Bs[kk][r] = (c0 + r < N && k < K) ? B[(c0 + r) * sbn + k * sbk] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
            for (int i = 0; i < 4; ++i) b[i] = Bs[kk][tx + 16 * i];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[i][q] = fma(a[i], b[q], acc[i][q]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t m = m0 + ty + 16 * i, c = c0 + tx + 16 * q;
            if (m < M && c < N) {
                double* p = C + m * ldc + c;
                *p = (beta == 0.0 ? 0.0 : beta * *p) + alpha * acc[i][q];
            }
        }
}

// tr(S), max S_jj, then S_jj += lambda with lambda = ridge_rel * tr(S) / d.
__global__ void ridge_kernel(double* S, int64_t d, double ridge_rel, double* out /*lambda, maxdiag*/) {
    __shared__ double st[256], sm[256];
    double t = 0.0, m = 0.0;
    for (int64_t j = threadIdx.x; j < d; j += 256) {
        const double v = S[j * d + j];
        t += v;
        m = fmax(m, v);
    }
    st[threadIdx.x] = t;
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            st[threadIdx.x] += st[threadIdx.x + o];
            sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
        }
        __syncthreads();
    }
    const double lam = ridge_rel * st[0] / (double)d;
    for (int64_t j = threadIdx.x; j < d; j += 256) S[j * d + j] += lam;
    if (threadIdx.x == 0) {
        out[0] = lam;
        out[1] = sm[0];
    }
}

// Unblocked Cholesky of the nb x nb diagonal block at (k0, k0); pivots recorded.  One
// thread per block entry: step p scales column p and updates T[r][c] (p < c <= r) once.
__global__ __launch_bounds__(kNB * kNB) void potrf_diag_kernel(double* A, int64_t d, int64_t k0, int nb,
                                                                double* pivots, int* bad) {
    __shared__ double T[kNB][kNB + 1];
    const int c = threadIdx.x % kNB, r = threadIdx.x / kNB;
    if (r < nb && c < nb) T[r][c] = A[(k0 + r) * d + k0 + c];
    __syncthreads();
    for (int p = 0; p < nb; ++p) {
        if (threadIdx.x == 0) {
            const double v = T[p][p];
            pivots[k0 + p] = v;
            if (!(v > 0.0)) *bad = 1;
            T[p][p] = v > 0.0 ? sqrt(v) : 1.0;
        }
        __syncthreads();
        if (c == p && r > p && r < nb) T[r][p] /= T[p][p];
        __syncthreads();
        if (c > p && c <= r && r < nb) T[r][c] -= T[r][p] * T[c][p];
        __syncthreads();
    }
    if (r < nb && c < nb) A[(k0 + r) * d + k0 + c] = c <= r ? T[r][c] : 0.0;
}

// Diagonal metric: the factor is diag(sqrt(S_jj + lambda)) (standardise, do not decorrelate).
__global__ void diag_factor_kernel(double* A, int64_t d, double* pivots, int* bad) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < d; j += (int64_t)gridDim.x * blockDim.x) {
        const double v = A[j * d + j];
        pivots[j] = v;
        if (!(v > 0.0)) *bad = 1;
        for (int64_t c = 0; c < d; ++c) A[j * d + c] = c == j ? (v > 0.0 ? sqrt(v) : 1.0) : 0.0;
    }
}

// Rows r0..r0+rows-1 of the nb-column block at column k0 of Mtx (leading dim ldm) are
// replaced by x with x L11^T = row, L11 the nb x nb lower block of L at (k0, k0).  One thread
// per row, the row held in registers (the loops unroll over the block size).
__global__ __launch_bounds__(128) void trsm_rows_kernel(double* Mtx, int64_t ldm, int64_t r0, int64_t rows,
                                                        int64_t col0, const double* L, int64_t d, int64_t k0,
                                                        int nb) {
    __shared__ double T[kNB][kNB + 1];
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) T[e / nb][e % nb] = L[(k0 + e / nb) * d + k0 + e % nb];
    __syncthreads();
    const int64_t r = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= r0 + rows) return;
    double* row = Mtx + r * ldm + col0;
    double x[kNB];
#pragma unroll
    for (int p = 0; p < kNB; ++p) x[p] = p < nb ? row[p] : 0.0;
#pragma unroll
    for (int p = 0; p < kNB; ++p) {
        if (p < nb) {
            double v = x[p];
#pragma unroll
            for (int t = 0; t < p; ++t) v -= x[t] * T[p][t];
            x[p] = v / T[p][p];
        }
    }
#pragma unroll
    for (int p = 0; p < kNB; ++p)
        if (p < nb) row[p] = x[p];
}

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float bf16_to_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Operand records.  Record (k, cb) (index k * ncb + cb) covers units 16k..16k+15 and
// covariates 32cb..32cb+31 in 2 planes of 64 lanes x 16 bytes; lane l = c + 32h:
//   split: plane 0 = BF16 hi, plane 1 = BF16 lo; dword t of lane l holds units
//          u = 32 (k / 2) + 8 (k % 2) + 4h + t (low half) and u + 16 (high half), so that
//          the contraction finds both bits of a dword 16 apart in a bitmask word;
//   fp32:  plane p holds X~(16k + 8p + 2q + h, 32cb + c), q = 0..3.
__global__ void operands_kernel(const double* X, int64_t n, int64_t d, int64_t ks, int64_t ncb,
                                uint4* op_split, uint4* op_f32) {
    const int64_t rec = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t k = rec / ncb, cb = rec % ncb;
    const int c = lane & 31, h = lane >> 5;
    const int64_t col = 32 * cb + c;
    auto x = [&](int64_t unit) -> double {
        return (unit < n && col < d) ? X[unit * d + col] : 0.0;
    };
    uint32_t hi[4], lo[4];
    for (int e = 0; e < 8; e += 2) {
        uint16_t hv[2], lv[2];
        for (int q = 0; q < 2; ++q) {
            const double v = x(32 * (k >> 1) + 8 * (k & 1) + 4 * h + e / 2 + 16 * q);
            const uint16_t hb = bf16_rne((float)v);
            const double r = v - (double)bf16_to_float(hb);
            hv[q] = hb;
            lv[q] = bf16_rne((float)r);
        }
        hi[e / 2] = (uint32_t)hv[0] | ((uint32_t)hv[1] << 16);
        lo[e / 2] = (uint32_t)lv[0] | ((uint32_t)lv[1] << 16);
    }
    op_split[rec * kRecordU4 + lane] = make_uint4(hi[0], hi[1], hi[2], hi[3]);
    op_split[rec * kRecordU4 + 64 + lane] = make_uint4(lo[0], lo[1], lo[2], lo[3]);
    if (!op_f32) return;
    for (int p = 0; p < 2; ++p) {
        float f[4];
        for (int q = 0; q < 4; ++q) f[q] = (float)x(16 * k + 8 * p + 2 * q + h);
        op_f32[rec * kRecordU4 + 64 * p + lane] =
            make_uint4(__float_as_uint(f[0]), __float_as_uint(f[1]), __float_as_uint(f[2]), __float_as_uint(f[3]));
    }
}

// Fixed-point form.  Block cb of 32 covariates gets the scale s = max |X~| / kQMax over its
// entries (rounded up to float, 1 for an all-zero block), so every entry quantises to
// q = rint(x / s) in [kQMin, kQMax]; q = 128 hi + lo with hi = floor((q + 64) / 128).
__global__ void block_scale_kernel(const double* X, int64_t n, int64_t d, float* bscale) {
    __shared__ double red[256];
    const int64_t cb = blockIdx.x;
    double m = 0.0;
    for (int64_t e = threadIdx.x; e < n * 32; e += blockDim.x) {
        const int64_t i = e / 32, col = 32 * cb + e % 32;
        if (col < d) m = fmax(m, fabs(X[i * d + col]));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double s = red[0] / (double)kQMax;
        float f = (float)s;
        if ((double)f < s) f = nextafterf(f, INFINITY);
        bscale[cb] = red[0] > 0.0 ? f : 1.0f;
    }
}

__device__ __forceinline__ int quantise(double x, float s) {
    const double q = fmin(fmax(rint(x / (double)s), (double)kQMin), (double)kQMax);
    return (int)q;
}

// Record (k, cb) of the fixed-point form: lane l = c + 32h holds, for t = 0..7, the digits of
// unit u = 16k + 8h + t and covariate 32cb + c in bytes 2t (-hi) and 2t + 1 (lo).  The
// contraction pairs them with the bytes -128 and 1 of a treated unit (0 otherwise), so one
// int8 MFMA K step of 32 sums 16 units' 128 hi + lo exactly.
__global__ void operands_i8_kernel(const double* X, int64_t n, int64_t d, int64_t ncb, const float* bscale,
                                   uint4* op_i8) {
    const int64_t rec = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t k = rec / ncb, cb = rec % ncb;
    const int c = lane & 31, h = lane >> 5;
    const int64_t col = 32 * cb + c;
    const float s = bscale[cb];
    uint32_t w[4];
    for (int t2 = 0; t2 < 4; ++t2) {
        uint32_t v = 0;
        for (int q2 = 0; q2 < 2; ++q2) {
            const int64_t unit = 16 * k + 8 * h + 2 * t2 + q2;
            const int q = (unit < n && col < d) ? quantise(X[unit * d + col], s) : 0;
            const int hi = (q + 64) >> 7;   // floor division (arithmetic shift)
            const int lo = q - 128 * hi;
            v |= (((uint32_t)(uint8_t)(int8_t)(-hi)) | ((uint32_t)(uint8_t)(int8_t)lo << 8)) << (16 * q2);
        }
        w[t2] = v;
    }
    op_i8[rec * kRecordU4I8 + lane] = make_uint4(w[0], w[1], w[2], w[3]);
}

// e_j = max(sum of the positive, sum of the negative parts of s q_ij - x_ij) over all units
// bounds |sum_{i in T} (s q_ij - x_ij)| for every treated set T; FP64, widened by 1e-12.
__global__ __launch_bounds__(kColW * kRowW) void qerr_kernel(const double* X, int64_t n, int64_t d,
                                                              const float* bscale, double* e) {
    __shared__ double part[2][kRowW][kColW];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * kColW + l;
    double v[2] = {0.0, 0.0}, t[2];
    if (j < d) {
        const float s = bscale[j / 32];
        for (int64_t i = w; i < n; i += kRowW) {
            const double x = X[i * d + j];
            const double r = (double)s * (double)quantise(x, s) - x;
            if (r > 0) v[0] += r; else v[1] -= r;
        }
    }
    combine_rows<2>(part, v, t);
    if (j < d && w == 0) e[j] = fmax(t[0], t[1]) * (1.0 + 1e-12);
}

// cabs_j = sum_i |X~_ij| rounded up to float; 0 for padded columns.
__global__ __launch_bounds__(kColW * kRowW) void cabs_kernel(const double* X, int64_t n, int64_t d, int64_t dpad,
                                                              float* cabs) {
    __shared__ double part[1][kRowW][kColW];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * kColW + l;
    double v[1] = {0.0}, t[1];
    if (j < d)
        for (int64_t i = w; i < n; i += kRowW) v[0] += fabs(X[i * d + j]);
    combine_rows<1>(part, v, t);
    if (j >= dpad || w != 0) return;
    if (j >= d) {
        cabs[j] = 0.f;
        return;
    }
    const double s = t[0] * (1.0 + 1e-12);   // cover the FP64 rounding of the sum itself
    float f = (float)s;
    if ((double)f < s) f = nextafterf(f, INFINITY);
    cabs[j] = f;
}

// Per-column quantities behind the error bounds of the FP32 contractions (out[5 d]: five
// arrays of d, each sum rounded up):
//   [0] split: sum_i |x_ij| 4 (ks - k_i), unit i entering at K step k_i = 2 (i / 32) +
//       ((i % 16) >= 8) (the operand record layout) and passing through at most 4 (ks - k_i)
//       rounding steps (two MFMA halves per plane, two planes per K step);
//   [1] split: sum over K steps and MFMA halves of the largest |x_ij| of the half (half h of
//       step k holds units base + 4h + t and base + 16 + 4h + t, t < 4, base = 32 (k / 2) +
//       8 (k % 2)): the dropped bits of a half-sum are bounded by its largest product;
//   [2] split: max(sum of the positive, sum of the negative) residuals x - hi - lo: no treated
//       set sums to more than either;
//   [3] fp32: sum_i |x_ij| (ks - i / 16), the VALU running-total adds unit i passes through;
//   [4] fp32: max(sum of the positive, sum of the negative) residuals x - float(x).
__global__ __launch_bounds__(kColW * kRowW) void bound_sums_kernel(const double* X, int64_t n, int64_t d, int64_t ks,
                                                                    double* out) {
    __shared__ double part[7][kRowW][kColW];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * kColW + l;
    auto x = [&](int64_t i) -> double { return i < n ? X[i * d + j] : 0.0; };
    // wsplit, tsplit, rsp, rsn, wf, rfp, rfn
    double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, t[7];
    if (j < d) {
        for (int64_t i = w; i < n; i += kRowW) {
            const double xv = x(i), a = fabs(xv);
            const int64_t ki = 2 * (i / 32) + ((i % 16) >= 8 ? 1 : 0);
            v[0] += a * (double)(4 * (ks - ki));
            v[4] += a * (double)(ks - i / 16);
            // the operand records' hi / lo: exact differences in FP64
            const double hi = (double)bf16_to_float(bf16_rne((float)xv));
            const double r1 = xv - hi;
            const double r = r1 - (double)bf16_to_float(bf16_rne((float)r1));
            if (r > 0) v[2] += r; else v[3] -= r;
            const double rf = xv - (double)(float)xv;
            if (rf > 0) v[5] += rf; else v[6] -= rf;
        }
        for (int64_t k = w; k < ks; k += kRowW) {
            const int64_t base = 32 * (k / 2) + 8 * (k % 2);
            for (int h = 0; h < 2; ++h) {
                double m = 0.0;
                for (int q = 0; q < 4; ++q)
                    m = fmax(m, fmax(fabs(x(base + 4 * h + q)), fabs(x(base + 16 + 4 * h + q))));
                v[1] += m;
            }
        }
    }
    combine_rows<7>(part, v, t);
    if (j >= d || w != 0) return;
    const double up = 1.0 + 1e-12;   // cover the FP64 rounding of the sums
    out[j] = t[0] * up;
    out[d + j] = t[1] * up;
    out[2 * d + j] = fmax(t[2], t[3]) * up;
    out[3 * d + j] = t[4] * up;
    out[4 * d + j] = fmax(t[5], t[6]) * up;
}

static hipError_t gemm_nt(hipStream_t st, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                          int64_t sam, int64_t sak, const double* B, int64_t sbn, int64_t sbk, double beta,
                          double* C, int64_t ldc) {
    if (M <= 0 || N <= 0) return hipSuccess;
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
    hipLaunchKernelGGL(dgemm_nt_kernel, grid, dim3(256), 0, st, M, N, K, alpha, A, sam, sak, B, sbn, sbk, beta, C, ldc);
    return hipGetLastError();
}

int pow2_chunks(int n);

rr_status prepare_impl(const void* dX, int x_dtype, int64_t n, int64_t d, int64_t ldx, int64_t n1,
                       double ridge_rel, int metric, hipStream_t st, rr_problem** out) {
    if (!dX || !out || n < 2 || d < 1 || ldx < d || n1 < 1 || n1 > n - 1 || !(ridge_rel >= 0.0) ||
        (x_dtype != RR_X_FP64 && x_dtype != RR_X_FP32) ||
        (metric != RR_METRIC_MAHALANOBIS && metric != RR_METRIC_DIAGONAL && metric != RR_METRIC_MAX_SMD)) {
        set_error("rr_prepare: invalid argument");
        return RR_E_ARG;
    }
    if (n > RR_MAX_N) {
        set_error("rr_prepare: n exceeds RR_MAX_N");
        return RR_E_UNSUPPORTED;
    }
    if (d > RR_MAX_D) {
        set_error("rr_prepare: d exceeds RR_MAX_D");
        return RR_E_UNSUPPORTED;
    }
    int device = 0;
    RR_HIP(hipGetDevice(&device));   // before the handle exists: nothing to release on failure
    static std::atomic<uint64_t> next_uid{1};
    auto* h = new rr_problem();
    Problem& P = h->P;
    P.device = device;
    P.uid = next_uid.fetch_add(1);
    P.n = n;
    P.d = d;
    P.n1 = n1;
    P.n0 = n - n1;
    P.ridge_rel = ridge_rel;
    P.metric = metric;
    P.S = pow2_chunks((int)n);
    P.wstride = 8 * P.S;
    P.ks = kKStepsPerStage * ((n + kKStepsPerStage * kKStep - 1) / (kKStepsPerStage * kKStep));  // whole LDS stages
    const int64_t cbq = 2;   // covariate blocks per contraction chunk
    P.ncb = (((d + kColBlock - 1) / kColBlock + cbq - 1) / cbq) * cbq;
    P.scale = (double)n / ((double)n1 * (double)(n - n1));
    const int64_t dpad = 32 * P.ncb;

    double *piv = nullptr, *scal = nullptr, *qe = nullptr;
    int* bad = nullptr;
    void* tmp = nullptr;   // qe, piv, scal and bad: one allocation for the call
    auto fail = [&](rr_status s) {
        hipFree(tmp);
        rr_free(h);
        return s;
    };
#define RR_PHIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            set_error(std::string("rr_prepare: ") + #call + ": " + hipGetErrorString(e_)); \
            return fail(RR_E_DEVICE);                                                     \
        }                                                                                 \
    } while (0)
    {
        // the handle's buffers in one allocation (and the call's temporaries in another): a
        // prepare of a small problem is otherwise dominated by allocator calls
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t o = off;
            off += (bytes + 255) & ~size_t(255);
            return o;
        };
        const size_t o_x = take(sizeof(double) * (n * d + kX64Pad)), o_l = take(sizeof(double) * d * d),
                     o_mu = take(sizeof(double) * d), o_sp = take(sizeof(uint4) * kRecordU4 * P.ks * P.ncb),
                     o_f32 = take(sizeof(uint4) * kRecordU4 * P.ks * P.ncb), o_cabs = take(sizeof(float) * dpad),
                     o_i8 = take(sizeof(uint4) * kRecordU4I8 * P.ks * P.ncb), o_bs = take(sizeof(float) * P.ncb);
        RR_PHIP(hipMalloc(&P.mem, off));
        char* b = static_cast<char*>(P.mem);
        P.X64 = reinterpret_cast<double*>(b + o_x);
        P.L = reinterpret_cast<double*>(b + o_l);
        P.mu = reinterpret_cast<double*>(b + o_mu);
        P.op_split = reinterpret_cast<uint4*>(b + o_sp);
        P.op_f32 = reinterpret_cast<uint4*>(b + o_f32);
        P.cabs = reinterpret_cast<float*>(b + o_cabs);
        P.op_i8 = reinterpret_cast<uint4*>(b + o_i8);
        P.bscale = reinterpret_cast<float*>(b + o_bs);
        off = 0;
        const size_t o_qe = take(sizeof(double) * 6 * d),   // e_j, then the five bound sums
            o_piv = take(sizeof(double) * d), o_scal = take(sizeof(double) * 2), o_bad = take(sizeof(int));
        RR_PHIP(hipMalloc(&tmp, off));
        char* t = static_cast<char*>(tmp);
        qe = reinterpret_cast<double*>(t + o_qe);
        piv = reinterpret_cast<double*>(t + o_piv);
        scal = reinterpret_cast<double*>(t + o_scal);
        bad = reinterpret_cast<int*>(t + o_bad);
    }
    RR_PHIP(hipMemsetAsync(P.X64 + n * d, 0, sizeof(double) * kX64Pad, st));
    RR_PHIP(hipMemsetAsync(bad, 0, sizeof(int), st));

    hipLaunchKernelGGL(mean_center_kernel, dim3((unsigned)((d + kColW - 1) / kColW)), dim3(kColW * kRowW), 0, st, dX,
                       x_dtype, n, d, ldx, P.mu, P.X64);
    RR_PHIP(hipGetLastError());
    // S = Xc^T Xc / (n - 1) into L's buffer, then factor in place.
    double* A = P.L;
    RR_PHIP(gemm_nt(st, d, d, n, 1.0 / (double)(n - 1), P.X64, 1, d, P.X64, 1, d, 0.0, A, d));
    hipLaunchKernelGGL(ridge_kernel, dim3(1), dim3(256), 0, st, A, d, ridge_rel, scal);
    RR_PHIP(hipGetLastError());
    if (metric != RR_METRIC_MAHALANOBIS) {
        hipLaunchKernelGGL(diag_factor_kernel, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, st, A, d, piv, bad);
        RR_PHIP(hipGetLastError());
    }
    for (int64_t k0 = 0; k0 < d && metric == RR_METRIC_MAHALANOBIS; k0 += kNB) {
        const int nb = (int)std::min<int64_t>(kNB, d - k0);
        hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(kNB * kNB), 0, st, A, d, k0, nb, piv, bad);
        RR_PHIP(hipGetLastError());
        const int64_t r0 = k0 + nb, rows = d - r0;
        if (rows > 0) {
            hipLaunchKernelGGL(trsm_rows_kernel, dim3((unsigned)((rows + 127) / 128)), dim3(128), 0, st, A, d, r0,
                               rows, k0, A, d, k0, nb);
            RR_PHIP(hipGetLastError());
            RR_PHIP(gemm_nt(st, rows, rows, nb, -1.0, A + r0 * d + k0, d, 1, A + r0 * d + k0, d, 1, 1.0,
                            A + r0 * d + r0, d));
        }
    }
    double hs[2];
    std::vector<double> hp((size_t)d);
    int hbad = 0;
    RR_PHIP(hipMemcpyAsync(hs, scal, sizeof(hs), hipMemcpyDeviceToHost, st));
    RR_PHIP(hipMemcpyAsync(hp.data(), piv, sizeof(double) * d, hipMemcpyDeviceToHost, st));
    RR_PHIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    RR_PHIP(hipStreamSynchronize(st));
    P.lambda = hs[0];
    double minpiv = INFINITY;
    for (double v : hp) minpiv = std::min(minpiv, v);
    if (hbad || !(minpiv >= 1e-10 * hs[1])) {
        set_error("rr_prepare: covariance is singular (use ridge_rel > 0)");
        return fail(RR_E_SINGULAR);
    }
    // upper triangle of L to zero (the factor is lower triangular)
    // X~ = Xc L^-T by column blocks, right-looking: solve block J with L[J, J], then
    // X[:, >J] -= X~[:, J] L[>J, J]^T (wide updates of depth nb).
    for (int64_t j0 = 0; j0 < d; j0 += kNB) {
        const int nb = (int)std::min<int64_t>(kNB, d - j0);
        hipLaunchKernelGGL(trsm_rows_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, P.X64, d, 0, n,
                           j0, A, d, j0, nb);
        RR_PHIP(hipGetLastError());
        const int64_t rest = d - j0 - nb;
        if (rest > 0)
            RR_PHIP(gemm_nt(st, n, rest, nb, -1.0, P.X64 + j0, d, 1, A + (j0 + nb) * d + j0, d, 1, 1.0,
                            P.X64 + j0 + nb, d));
    }
    hipLaunchKernelGGL(operands_kernel, dim3((unsigned)(P.ks * P.ncb)), dim3(64), 0, st, P.X64, n, d, P.ks, P.ncb,
                       P.op_split, P.op_f32);
    RR_PHIP(hipGetLastError());
    hipLaunchKernelGGL(cabs_kernel, dim3((unsigned)((dpad + kColW - 1) / kColW)), dim3(kColW * kRowW), 0, st, P.X64,
                       n, d, dpad, P.cabs);
    RR_PHIP(hipGetLastError());
    hipLaunchKernelGGL(block_scale_kernel, dim3((unsigned)P.ncb), dim3(256), 0, st, P.X64, n, d, P.bscale);
    RR_PHIP(hipGetLastError());
    hipLaunchKernelGGL(operands_i8_kernel, dim3((unsigned)(P.ks * P.ncb)), dim3(64), 0, st, P.X64, n, d, P.ncb,
                       P.bscale, P.op_i8);
    RR_PHIP(hipGetLastError());
    hipLaunchKernelGGL(qerr_kernel, dim3((unsigned)((d + kColW - 1) / kColW)), dim3(kColW * kRowW), 0, st, P.X64, n,
                       d, P.bscale, qe);
    RR_PHIP(hipGetLastError());
    hipLaunchKernelGGL(bound_sums_kernel, dim3((unsigned)((d + kColW - 1) / kColW)), dim3(kColW * kRowW), 0, st,
                       P.X64, n, d, P.ks, qe + d);
    RR_PHIP(hipGetLastError());
    {
        std::vector<float> hc((size_t)dpad);
        std::vector<double> he((size_t)(6 * d));
        RR_PHIP(hipMemcpyAsync(hc.data(), P.cabs, sizeof(float) * dpad, hipMemcpyDeviceToHost, st));
        RR_PHIP(hipMemcpyAsync(he.data(), qe, sizeof(double) * 6 * d, hipMemcpyDeviceToHost, st));
        RR_PHIP(hipStreamSynchronize(st));
        double c2 = 0.0, cmax = 0.0;
        for (float c : hc) {
            c2 += (double)c * (double)c;
            cmax = std::max(cmax, (double)c);
        }
        P.cabs_c2 = c2;
        P.cabs_max = cmax;
        double e2 = 0.0, emax = 0.0;
        for (int64_t j = 0; j < d; ++j) {
            e2 += he[j] * he[j];
            emax = std::max(emax, he[j]);
        }
        P.qerr_c2 = e2 * (1.0 + 1e-12);
        P.qerr_max = emax;
        // per-column bounds of |G32_j - G_j| of the split and FP32 contractions (rounding model
        // and constants in bound_constants)
        std::vector<double> es((size_t)d), ef((size_t)d);
        for (int64_t j = 0; j < d; ++j) {
            es[j] = split_column_bound(P, he[d + j], he[2 * d + j], he[3 * d + j]);
            ef[j] = fp32_column_bound(P, (double)hc[j], he[4 * d + j], he[5 * d + j]);
        }
        auto norm2 = [](const std::vector<double>& v) {
            double s2 = 0.0, m = 0.0;
            for (double x : v) {
                s2 += x * x;
                m = std::max(m, x);
            }
            return std::make_pair(s2 * (1.0 + 1e-12), m);
        };
        std::tie(P.esplit_n2, P.esplit_max) = norm2(es);
        std::tie(P.ef32_n2, P.ef32_max) = norm2(ef);
    }
    hipFree(tmp);
    tmp = nullptr;
    // the device's binomial table (exact-mode keys), so that later calls find it without allocating
    if (!binom_table(device)) {
        set_error("rr_prepare: binomial table allocation failed");
        return fail(RR_E_DEVICE);
    }
#undef RR_PHIP
    *out = h;
    return RR_OK;
}

// Gram form: K = X~ X~^T (n x n, FP64), its split operand records with K's columns in the
// place of the covariates (K is symmetric), and the error-bound constant sum of the n1
// largest column sums of |K|.
rr_status ensure_gram(Problem& P, hipStream_t st) {
    if (P.op_gram) return RR_OK;
    const int64_t n = P.n, d = P.d;
    const int64_t cbq = 2;
    const int64_t ncb = cbq * ((n + 32 * cbq - 1) / (32 * cbq));
    const int64_t npad = 32 * ncb;
    double* K = nullptr;
    float* cabs = nullptr;
    uint4* op = nullptr;
    auto fail = [&](hipError_t e) {
        hipFree(K);
        hipFree(cabs);
        hipFree(op);
        set_error(std::string("rr_draw: Gram operands: ") + hipGetErrorString(e));
        return RR_E_DEVICE;
    };
    hipError_t e = hipMalloc(&K, sizeof(double) * n * n);
    if (e == hipSuccess) e = hipMalloc(&cabs, sizeof(float) * npad);
    if (e == hipSuccess) e = hipMalloc(&op, sizeof(uint4) * kRecordU4 * P.ks * ncb);
    if (e != hipSuccess) return fail(e);
    e = gemm_nt(st, n, n, d, 1.0, P.X64, d, 1, P.X64, d, 1, 0.0, K, n);
    if (e != hipSuccess) return fail(e);
    hipLaunchKernelGGL(operands_kernel, dim3((unsigned)(P.ks * ncb)), dim3(64), 0, st, K, n, n, P.ks, ncb, op,
                       (uint4*)nullptr);
    hipLaunchKernelGGL(cabs_kernel, dim3((unsigned)((npad + kColW - 1) / kColW)), dim3(kColW * kRowW), 0, st, K, n, n,
                       npad, cabs);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e);
    std::vector<float> hc((size_t)npad);
    if ((e = hipMemcpyAsync(hc.data(), cabs, sizeof(float) * npad, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return fail(e);
    std::sort(hc.begin(), hc.end(), [](float x, float y) { return x > y; });
    double top = 0.0;
    for (int64_t i = 0; i < P.n1 && i < npad; ++i) top += (double)hc[i];
    hipFree(K);
    hipFree(cabs);
    P.op_gram = op;
    P.ncb_gram = ncb;
    P.gram_ctop = top * (1.0 + 1e-12);
    return RR_OK;
}

}  // namespace rr
