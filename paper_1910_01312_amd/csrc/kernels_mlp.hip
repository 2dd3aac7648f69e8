// Warm-start network kernels (fp32): the 66 -> 256 -> 256 -> 4 GELU network
// that predicts, per sample, whether x_i* is 0, inside (0, C) or C, and
// x_i*/C when inside; its loss, gradients and Adam update; and the feature
// and initial-point kernels around it.
//
// All matrix products go through one LDS-tiled GEMM
//     C[M x N] = op(A)[M x K] op(B)[K x N]      (row-major operands)
// with 64 x 64 output tiles, K staged 16 at a time, 4 x 4 outputs per thread
// and fused epilogues (bias, bias + GELU keeping the pre-activation,
// multiplication by GELU'(pre)).  Weight gradients (K = batch rows) use a
// fixed split of K with one partial tile per split, reduced in split order:
// deterministic.
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {

constexpr int GT = 64;             // output tile
constexpr int GK = 16;             // K slice staged in LDS

__device__ __forceinline__ float gelu_f(float a) {
    return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float a) {
    return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) +
           a * expf(-0.5f * a * a) * 0.39894228040143268f;
}

enum { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_GRAD = 3 };

// C (or the split partial) = op(A) op(B) over K range of split blockIdx.z.
// EPI_BIAS_GELU writes pre = acc + bias to C and gelu(pre) to C2;
// EPI_GELU_GRAD writes acc * gelu'(E[m][n]) to C.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(const float* __restrict__ A, int lda,
                                              const float* __restrict__ B, int ldb,
                                              float* __restrict__ C, float* __restrict__ C2, int ldc,
                                              const float* __restrict__ bias,
                                              const float* __restrict__ E,
                                              int M, int N, int K, int kchunk,
                                              float* __restrict__ part) {
    __shared__ float As[GK][GT + 4];
    __shared__ float Bs[GK][GT + 4];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int k0 = blockIdx.z * kchunk, k1 = min(K, k0 + kchunk);
    float acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0f;
    for (int kb = k0; kb < k1; kb += GK) {
        // stage op(A)[m0:m0+64][kb:kb+16] and op(B)[kb:kb+16][n0:n0+64]
        for (int e = threadIdx.x; e < GK * GT; e += 256) {
            int kk, mm;
            if (TA) { mm = e % GT; kk = e / GT; }          // A stored K x M: rows of K contiguous in m
            else { kk = e % GK; mm = e / GK; }              // A stored M x K
            const int m = m0 + mm, k = kb + kk;
            float v = 0.0f;
            if (m < M && k < k1) v = TA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k];
            As[kk][mm] = v;
        }
        for (int e = threadIdx.x; e < GK * GT; e += 256) {
            int kk, nn;
            if (TB) { kk = e % GK; nn = e / GK; }          // B stored N x K
            else { nn = e % GT; kk = e / GT; }              // B stored K x N
            const int nidx = n0 + nn, k = kb + kk;
            float v = 0.0f;
            if (nidx < N && k < k1) v = TB ? B[(int64_t)nidx * ldb + k] : B[(int64_t)k * ldb + nidx];
            Bs[kk][nn] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = As[kk][ty * 4 + u];
                b[u] = Bs[kk][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(a[u], b[v], acc[u][v]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int m = m0 + ty * 4 + u;
        if (m >= M) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int nidx = n0 + tx * 4 + v;
            if (nidx >= N) continue;
            const float r = acc[u][v];
            if (part) {
                part[((int64_t)blockIdx.z * M + m) * N + nidx] = r;
            } else if (EPI == EPI_BIAS) {
                C[(int64_t)m * ldc + nidx] = r + bias[nidx];
            } else if (EPI == EPI_BIAS_GELU) {
                const float pre = r + bias[nidx];
                C[(int64_t)m * ldc + nidx] = pre;
                C2[(int64_t)m * ldc + nidx] = gelu_f(pre);
            } else if (EPI == EPI_GELU_GRAD) {
                C[(int64_t)m * ldc + nidx] = r * gelu_grad_f(E[(int64_t)m * ldc + nidx]);
            } else {
                C[(int64_t)m * ldc + nidx] = r;
            }
        }
    }
}

// C[i] = sum over splits of part[z][i] (split order)
__global__ __launch_bounds__(256) void k_split_reduce(const float* __restrict__ part, int nsplit,
                                                      int64_t count, float* __restrict__ C) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.0f;
    for (int z = 0; z < nsplit; ++z) s += part[(int64_t)z * count + i];
    C[i] = s;
}

// db[c] = sum over rows of D[r][c] (64 columns per block, 4 row groups, fixed order)
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ D, int n, int N,
                                                float* __restrict__ db) {
    __shared__ float sh[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
    float s = 0.0f;
    if (c < N)
        for (int r = g; r < n; r += 4) s += D[(int64_t)r * N + c];
    sh[g][threadIdx.x & 63] = s;
    __syncthreads();
    if (g == 0 && c < N) db[c] = (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
}

// head: out[i] = (softmax(O[i,0:3]), sigmoid(O[i,3]))
__global__ __launch_bounds__(256) void k_head(const float* __restrict__ O, int64_t n,
                                              float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 o = *reinterpret_cast<const float4*>(O + 4 * i);
    const float mx = fmaxf(o.x, fmaxf(o.y, o.z));
    const float e0 = expf(o.x - mx), e1 = expf(o.y - mx), e2 = expf(o.z - mx);
    const float inv = 1.0f / (e0 + e1 + e2);
    float4 r;
    r.x = e0 * inv;
    r.y = e1 * inv;
    r.z = e2 * inv;
    r.w = 1.0f / (1.0f + expf(-o.w));
    *reinterpret_cast<float4*>(out + 4 * i) = r;
}

// loss terms and dL/dO for the mean loss over n rows:
//   -log P[s] + w [s == 1] (mult - t)^2;  dO = (P - onehot(s), [s==1] 2 w (mult - t) mult (1 - mult)) / n
// per-block loss partials (fixed order inside the block)
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ out,
                                              const int32_t* __restrict__ st,
                                              const float* __restrict__ tg, int64_t n, float w,
                                              float* __restrict__ dO, double* __restrict__ lpart) {
    __shared__ double sh[SSN_WAVES_PER_BLOCK];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (i < n) {
        const float4 o = *reinterpret_cast<const float4*>(out + 4 * i);
        const int s = st[i];
        const float t = tg[i];
        const float inside = s == 1 ? 1.0f : 0.0f;
        const float ps = s == 0 ? o.x : (s == 1 ? o.y : o.z);
        const float dm = o.w - t;
        l = -log((double)ps) + (double)(w * inside * dm * dm);
        const float invn = 1.0f / (float)n;
        float4 d;
        d.x = (o.x - (s == 0 ? 1.0f : 0.0f)) * invn;
        d.y = (o.y - (s == 1 ? 1.0f : 0.0f)) * invn;
        d.z = (o.z - (s == 2 ? 1.0f : 0.0f)) * invn;
        d.w = inside * 2.0f * w * dm * o.w * (1.0f - o.w) * invn;
        *reinterpret_cast<float4*>(dO + 4 * i) = d;
    }
    const double b = block_sum(l, sh);
    if (threadIdx.x == 0) lpart[blockIdx.x] = b;
}
__global__ __launch_bounds__(256) void k_loss_fin(const double* __restrict__ lpart, int nb, int64_t n,
                                                  float* __restrict__ loss) {
    __shared__ double sh[SSN_WAVES_PER_BLOCK];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += lpart[b];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) *loss = (float)(s / (double)n);
}

// Adam (bias-corrected), elementwise over the flat parameter vector
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ th, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              int64_t count, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------ features
// Z[i][0:64] = X_i R (fp32 accumulation), Z[i][64] = (A w1)_i + y_i b1,
// Z[i][65] = lognc.  One block: 64 rows, 256 threads = 64 rows x 4 groups of
// 16 outputs; X rows and R staged in LDS by 32-column slices.
template <typename T>
__global__ __launch_bounds__(256) void k_ws_features(const T* __restrict__ X,
                                                     const int8_t* __restrict__ y, int64_t n, int q,
                                                     const float* __restrict__ R,
                                                     const double* __restrict__ aw, double b1,
                                                     float lognc, float* __restrict__ Z) {
    __shared__ float Xs[64][33];
    __shared__ float Rs[32][64];
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int rr = threadIdx.x & 63, g = threadIdx.x >> 6;
    float acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.0f;
    for (int c0 = 0; c0 < q; c0 += 32) {
        for (int e = threadIdx.x; e < 64 * 32; e += 256) {
            const int a = e / 32, b = e % 32;
            const int64_t r = r0 + a;
            const int c = c0 + b;
            Xs[a][b] = (r < n && c < q) ? (float)to_f64(X[r * q + c]) : 0.0f;
        }
        for (int e = threadIdx.x; e < 32 * 64; e += 256) {
            const int a = e / 64, b = e % 64;
            const int c = c0 + a;
            Rs[a][b] = c < q ? R[(int64_t)c * 64 + b] : 0.0f;
        }
        __syncthreads();
#pragma unroll 4
        for (int c = 0; c < 32; ++c) {
            const float xv = Xs[rr][c];
#pragma unroll
            for (int k = 0; k < 16; ++k) acc[k] = fmaf(xv, Rs[c][g * 16 + k], acc[k]);
        }
        __syncthreads();
    }
    const int64_t r = r0 + rr;
    if (r >= n) return;
    float* zr = Z + r * 66;
#pragma unroll
    for (int k = 0; k < 16; ++k) zr[g * 16 + k] = acc[k];
    if (g == 0) {
        zr[64] = (float)(aw[r] + (double)y[r] * b1);
        zr[65] = lognc;
    }
}

// class sums of (A w1)_i: part[b*4 + {0,1,2,3}] = (sum over y=+1, count +1,
// sum over y=-1, count -1) per block
__global__ __launch_bounds__(256) void k_class_sums(const double* __restrict__ aw,
                                                    const int8_t* __restrict__ y, int64_t n,
                                                    double* __restrict__ part) {
    __shared__ double sh[SSN_WAVES_PER_BLOCK];
    double sp = 0.0, cp = 0.0, sn = 0.0, cn = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        // s_i = x_i^T w1 = y_i (A w1)_i
        if (y[i] > 0) { sp += aw[i]; cp += 1.0; }
        else { sn -= aw[i]; cn += 1.0; }
    }
    const double a = block_sum(sp, sh), b = block_sum(cp, sh), c = block_sum(sn, sh), d = block_sum(cn, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 4 + 0] = a;
        part[blockIdx.x * 4 + 1] = b;
        part[blockIdx.x * 4 + 2] = c;
        part[blockIdx.x * 4 + 3] = d;
    }
}

// x0_i by the most probable status (ties to the lower index): 0, C mult, C
__global__ __launch_bounds__(256) void k_ws_x0(const float* __restrict__ out, int64_t n, double C,
                                               double* __restrict__ x0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 o = *reinterpret_cast<const float4*>(out + 4 * i);
    const int k = (o.y > o.x) ? ((o.z > o.y) ? 2 : 1) : ((o.z > o.x) ? 2 : 0);
    x0[i] = k == 0 ? 0.0 : (k == 1 ? C * (double)o.w : C);
}

// Training labels from a solution x: status 0 (x_i <= 1e-8 C), 2 (x_i >=
// (1 - 1e-8) C) or 1 (inside), and the multiplier target x_i / C.
__global__ __launch_bounds__(256) void k_ws_labels(const double* __restrict__ x, int64_t n, double C,
                                                   int32_t* __restrict__ status,
                                                   float* __restrict__ target) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = x[i];
    status[i] = xi >= (1.0 - 1e-8) * C ? 2 : (xi <= 1e-8 * C ? 0 : 1);
    target[i] = (float)(xi / C);
}

// ------------------------------------------------------------------ screening
// Xk[j] = X[list[j]], yk[j] = y[list[j]] (one row per 64 threads)
template <typename T>
__global__ __launch_bounds__(256) void k_gather_rows(const T* __restrict__ X,
                                                     const int8_t* __restrict__ y,
                                                     const int32_t* __restrict__ list, int64_t m,
                                                     int q, T* __restrict__ Xk,
                                                     int8_t* __restrict__ yk) {
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= m) return;
    const int64_t r = list[j];
    for (int c = lane; c < q; c += 64) Xk[j * q + c] = X[r * q + c];
    if (lane == 0) yk[j] = y[r];
}
// x[list[j]] = xk[j] (x cleared beforehand)
__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ list, int64_t m,
                                                 const double* __restrict__ xk,
                                                 double* __restrict__ x) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) x[list[j]] = xk[j];
}
// Histogram of s_i = -log10(1 - P0_i) over HBINS bins of [0, HMAX) (the
// last bin takes everything above): the rows most surely at x = 0 have the
// largest s.  Integer counts, so the result does not depend on the order.
constexpr int HBINS = 4096;
constexpr float HMAX = 8.0f;
__device__ __forceinline__ int p0_bin(float p0) {
    const float s = -log10f(fmaxf(1.0f - p0, 1e-30f));
    const int b = (int)(s * (HBINS / HMAX));
    return b < 0 ? 0 : (b >= HBINS ? HBINS - 1 : b);
}
__global__ __launch_bounds__(256) void k_p0_hist(const float* __restrict__ out, int64_t n,
                                                 unsigned* __restrict__ hist) {
    __shared__ unsigned h[HBINS];
    for (int i = threadIdx.x; i < HBINS; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[p0_bin(out[4 * i])], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < HBINS; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}
// keep[i] = 1 when the bin of row i is below cut (the rows left are those
// of bins >= cut)
__global__ __launch_bounds__(256) void k_ws_keep_bin(const float* __restrict__ out, int64_t n,
                                                     int cut, uint8_t* __restrict__ keep) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keep[i] = p0_bin(out[4 * i]) < cut ? 1 : 0;
}
// xk[j] = x[list[j]]
__global__ __launch_bounds__(256) void k_gather_vec(const double* __restrict__ x,
                                                    const int32_t* __restrict__ list, int64_t m,
                                                    double* __restrict__ xk) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) xk[j] = x[list[j]];
}
// add margin violators: keep[i] = 1 where y_i (w^T x_i + b) = (A w)_i + y_i b < 1
__global__ __launch_bounds__(256) void k_ws_violators(const double* __restrict__ aw,
                                                      const int8_t* __restrict__ y, int64_t n,
                                                      double b, uint8_t* __restrict__ keep) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (aw[i] + (double)y[i] * b < 1.0) keep[i] = 1;
}

__global__ void k_fill_u32(unsigned* __restrict__ p, int len) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) p[i] = 0u;
}

// ------------------------------------------------------------------ launchers
static inline dim3 ggrid(int M, int N, int nsplit) {
    return dim3((N + GT - 1) / GT, (M + GT - 1) / GT, nsplit);
}
#define GEMM(TA, TB, EPI, M, N, K, kchunk, nsplit, ...)                                        \
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), ggrid(M, N, nsplit), dim3(256), 0, s, __VA_ARGS__, \
                       M, N, K, kchunk, part)

int mlp_splits(int64_t n) {
    int s = (int)((n + 511) / 512);
    return s < 1 ? 1 : (s > 64 ? 64 : s);
}

void launch_mlp_forward(const float* th, const float* Zin, int64_t n, float* work, float* O,
                        float* out, hipStream_t s) {
    const int I = MLP_IN, H = MLP_HID, NO = MLP_OUT;
    const float *W1 = th, *b1 = W1 + I * H, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + H * NO;
    float* A1 = work;
    float* H1 = A1 + n * H;
    float* A2 = H1 + n * H;
    float* H2 = A2 + n * H;
    float* part = nullptr;
    const int M = (int)n;
    GEMM(false, false, EPI_BIAS_GELU, M, H, I, I, 1, Zin, I, W1, H, A1, H1, H, b1, nullptr);
    GEMM(false, false, EPI_BIAS_GELU, M, H, H, H, 1, H1, H, W2, H, A2, H2, H, b2, nullptr);
    GEMM(false, false, EPI_BIAS, M, NO, H, H, 1, H2, H, W3, NO, O, nullptr, NO, b3, nullptr);
    hipLaunchKernelGGL(k_head, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, O, n, out);
}

void launch_mlp_backward(const float* th, const float* Zin, int64_t n, const float* work,
                         const float* out, const int32_t* st, const float* tg, float w,
                         float* grad, float* loss, float* scratch, hipStream_t s) {
    const int I = MLP_IN, H = MLP_HID, NO = MLP_OUT;
    const float *W2 = th + I * H + H, *W3 = W2 + H * H + H;
    float *gW1 = grad, *gb1 = gW1 + I * H, *gW2 = gb1 + H, *gb2 = gW2 + H * H, *gW3 = gb2 + H,
          *gb3 = gW3 + H * NO;
    const float* A1 = work;
    const float* H1 = A1 + n * H;
    const float* A2 = H1 + n * H;
    const float* H2 = A2 + n * H;
    float* dO = scratch;                     // n x 4
    float* dA2 = dO + 4 * n;                 // n x H
    float* dA1 = dA2 + n * H;                // n x H
    float* pbuf = dA1 + n * H;               // splits x H x H
    double* lpart = reinterpret_cast<double*>(pbuf + (int64_t)64 * H * H);
    const int M = (int)n, nb = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, s, out, st, tg, n, w, dO, lpart);
    hipLaunchKernelGGL(k_loss_fin, dim3(1), dim3(256), 0, s, lpart, nb, n, loss);
    const int ns = mlp_splits(n);
    const int kc = (int)((n + ns - 1) / ns);
    float* part = pbuf;
    // layer 3: gW3 = H2^T dO, gb3 = colsum dO, dA2 = (dO W3^T) * gelu'(A2)
    GEMM(true, false, EPI_NONE, H, NO, M, kc, ns, H2, H, dO, NO, nullptr, nullptr, NO, nullptr, nullptr);
    hipLaunchKernelGGL(k_split_reduce, dim3((H * NO + 255) / 256), dim3(256), 0, s, pbuf, ns,
                       (int64_t)H * NO, gW3);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, s, dO, M, NO, gb3);
    part = nullptr;
    GEMM(false, true, EPI_GELU_GRAD, M, H, NO, NO, 1, dO, NO, W3, NO, dA2, nullptr, H, nullptr, A2);
    // layer 2
    part = pbuf;
    GEMM(true, false, EPI_NONE, H, H, M, kc, ns, H1, H, dA2, H, nullptr, nullptr, H, nullptr, nullptr);
    hipLaunchKernelGGL(k_split_reduce, dim3((H * H + 255) / 256), dim3(256), 0, s, pbuf, ns,
                       (int64_t)H * H, gW2);
    hipLaunchKernelGGL(k_colsum, dim3(H / 64), dim3(256), 0, s, dA2, M, H, gb2);
    part = nullptr;
    GEMM(false, true, EPI_GELU_GRAD, M, H, H, H, 1, dA2, H, W2, H, dA1, nullptr, H, nullptr, A1);
    // layer 1
    part = pbuf;
    GEMM(true, false, EPI_NONE, I, H, M, kc, ns, Zin, I, dA1, H, nullptr, nullptr, H, nullptr, nullptr);
    hipLaunchKernelGGL(k_split_reduce, dim3((I * H + 255) / 256), dim3(256), 0, s, pbuf, ns,
                       (int64_t)I * H, gW1);
    hipLaunchKernelGGL(k_colsum, dim3(H / 64), dim3(256), 0, s, dA1, M, H, gb1);
}

void launch_adam(float* th, const float* g, float* m, float* v, int64_t count, float lr, float b1,
                 float b2, float eps, int step, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, th, g, m, v,
                       count, lr, b1, b2, eps, c1, c2);
}

void launch_class_sums(const double* aw, const int8_t* y, int64_t n, double* part, int nb,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_class_sums, dim3(nb), dim3(256), 0, s, aw, y, n, part);
}

void launch_ws_features(int dtype, const void* X, const int8_t* y, int64_t n, int64_t q,
                        const float* R, const double* aw, double b1, float lognc, float* Z,
                        hipStream_t s) {
    const dim3 g((unsigned)((n + 63) / 64));
    if (dtype == SSNALM_F64)
        hipLaunchKernelGGL(k_ws_features<double>, g, dim3(256), 0, s, (const double*)X, y, n, (int)q, R,
                           aw, b1, lognc, Z);
    else if (dtype == SSNALM_F32)
        hipLaunchKernelGGL(k_ws_features<float>, g, dim3(256), 0, s, (const float*)X, y, n, (int)q, R,
                           aw, b1, lognc, Z);
    else
        hipLaunchKernelGGL(k_ws_features<bf16_t>, g, dim3(256), 0, s, (const bf16_t*)X, y, n, (int)q,
                           R, aw, b1, lognc, Z);
}

void launch_gather_rows(int dtype, const void* X, const int8_t* y, const int32_t* list, int64_t m,
                        int64_t q, void* Xk, int8_t* yk, hipStream_t s) {
    const dim3 g((unsigned)((m + 3) / 4));
    if (dtype == SSNALM_F64)
        hipLaunchKernelGGL(k_gather_rows<double>, g, dim3(256), 0, s, (const double*)X, y, list, m,
                           (int)q, (double*)Xk, yk);
    else if (dtype == SSNALM_F32)
        hipLaunchKernelGGL(k_gather_rows<float>, g, dim3(256), 0, s, (const float*)X, y, list, m,
                           (int)q, (float*)Xk, yk);
    else
        hipLaunchKernelGGL(k_gather_rows<bf16_t>, g, dim3(256), 0, s, (const bf16_t*)X, y, list, m,
                           (int)q, (bf16_t*)Xk, yk);
}
void launch_scatter(const int32_t* list, int64_t m, const double* xk, double* x, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, list, m, xk, x);
}
int p0_hist_bins() { return HBINS; }
void launch_p0_hist(const float* out, int64_t n, unsigned* hist, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3((HBINS + 255) / 256), dim3(256), 0, s, hist, HBINS);
    hipLaunchKernelGGL(k_p0_hist, dim3(256), dim3(256), 0, s, out, n, hist);
}
void launch_ws_keep_bin(const float* out, int64_t n, int cut, uint8_t* keep, hipStream_t s) {
    hipLaunchKernelGGL(k_ws_keep_bin, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, cut,
                       keep);
}
void launch_gather_vec(const double* x, const int32_t* list, int64_t m, double* xk, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_vec, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, x, list, m, xk);
}
void launch_ws_violators(const double* aw, const int8_t* y, int64_t n, double b, uint8_t* keep,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_ws_violators, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, aw, y, n, b,
                       keep);
}

void launch_ws_x0(const float* out, int64_t n, double C, double* x0, hipStream_t s) {
    hipLaunchKernelGGL(k_ws_x0, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, C, x0);
}
void launch_ws_labels(const double* x, int64_t n, double C, int32_t* status, float* target,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_ws_labels, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, C,
                       status, target);
}

}  // namespace ssn
