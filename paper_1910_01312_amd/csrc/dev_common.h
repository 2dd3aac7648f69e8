// Device helpers shared by the gfx950 kernels: wave64 reductions, element
// loads for fp64 / fp32 / bfloat16 storage, and the "last block finishes"
// grid reduction handshake used for deterministic two-stage reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SSN_WAVE 64
#define SSN_BLOCK 256
#define SSN_WAVES_PER_BLOCK (SSN_BLOCK / SSN_WAVE)

typedef uint16_t bf16_t;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = SSN_WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, SSN_WAVE);
    return v;
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
    for (int off = SSN_WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, SSN_WAVE);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = SSN_WAVE / 2; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, SSN_WAVE));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = SSN_WAVE / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, SSN_WAVE));
    return v;
}

// Sum over the block of one double per thread; result valid in every thread.
// Fixed combination order -> deterministic.
__device__ __forceinline__ double block_sum(double v, double* sh /* >= SSN_WAVES_PER_BLOCK */) {
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < SSN_WAVES_PER_BLOCK; ++i) r += sh[i];
    return r;
}
// K block sums at once with one pair of barriers (fixed order: waves in
// index order).  sh: K * SSN_WAVES_PER_BLOCK doubles of LDS.
template <int K>
__device__ __forceinline__ void block_sum_n(double (&v)[K], double* sh) {
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) sh[k * SSN_WAVES_PER_BLOCK + w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double r = 0.0;
#pragma unroll
        for (int i = 0; i < SSN_WAVES_PER_BLOCK; ++i) r += sh[k * SSN_WAVES_PER_BLOCK + i];
        v[k] = r;
    }
}
__device__ __forceinline__ long long block_sum_ll(long long v, long long* sh) {
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    v = wave_sum_ll(v);
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    long long r = 0;
#pragma unroll
    for (int i = 0; i < SSN_WAVES_PER_BLOCK; ++i) r += sh[i];
    return r;
}

// Returns true in every thread of the block that is the last one of the
// grid to arrive.  The caller must have written its partial results before
// calling.  The counter is reset by the last block so it can be reused by
// the next launch on the same stream.  Every wave first waits for its own
// stores to complete; then one thread per block makes them visible device
// wide (one agent-scope fence per block: a fence in every wave costs several
// times more on a multi-die device) and arrives.
__device__ __forceinline__ bool last_block_arrives(unsigned* counter) {
    __shared__ int s_last;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev = atomicAdd(counter, 1u);
        const int last = (prev == gridDim.x * gridDim.y * gridDim.z - 1) ? 1 : 0;
        if (last) {
            __threadfence();
            atomicExch(counter, 0u);
        }
        s_last = last;
    }
    __syncthreads();
    return s_last != 0;
}

// Load of a value that another block of the grid wrote before
// last_block_arrives (whose fences make it visible to the last block), or
// that an earlier kernel wrote: a plain load, so that the compiler can keep
// many of them in flight.
__device__ __forceinline__ double ld_grid(const double* p) { return *p; }
__device__ __forceinline__ long long ld_grid(const long long* p) { return *p; }
__device__ __forceinline__ int ld_grid(const int* p) { return *p; }

// Sum of column c of a partials array (part[b*stride + c], b < nb) by the
// whole block: thread t sums b = t, t+blockDim, ... with four independent
// accumulators (loads in flight), then a fixed-order block reduction.  The
// mapping from b to thread and the combination order are fixed, so the
// result is deterministic.  Every thread of the block must call it.
__device__ __forceinline__ double grid_colsum(const double* part, int nb, int stride, int c,
                                              double* sh) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    const int T = blockDim.x;
    int b = threadIdx.x;
    for (; b + 3 * T < nb; b += 4 * T) {
        a0 += ld_grid(&part[(int64_t)b * stride + c]);
        a1 += ld_grid(&part[(int64_t)(b + T) * stride + c]);
        a2 += ld_grid(&part[(int64_t)(b + 2 * T) * stride + c]);
        a3 += ld_grid(&part[(int64_t)(b + 3 * T) * stride + c]);
    }
    for (; b < nb; b += T) a0 += ld_grid(&part[(int64_t)b * stride + c]);
    return block_sum((a0 + a1) + (a2 + a3), sh);
}

// Reduce-scatter over the wave: on entry every lane holds a[0..63]; on exit
// lane l returns the wave total of a[l].  At each step lanes paired by
// xor h keep one half of their live values (the upper half if bit h is set)
// and add the partner's copy of that half: 63 exchanges instead of 64 full
// wave sums, in a fixed order.
__device__ __forceinline__ double wave_reduce_scatter64(double (&a)[64]) {
    const int lane = threadIdx.x & (SSN_WAVE - 1);
#pragma unroll
    for (int h = 32; h >= 1; h >>= 1) {
        const bool up = (lane & h) != 0;
#pragma unroll
        for (int j = 0; j < h; ++j) {
            const double lo_v = a[j], hi_v = a[j + h];
            const double send = up ? lo_v : hi_v;
            const double keep = up ? hi_v : lo_v;
            a[j] = keep + __shfl_xor(send, h, SSN_WAVE);
        }
    }
    return a[0];
}

// block_append for U values per thread (value u of thread t is element
// u * blockDim + t): one pair of barriers for all U, list order = element order
template <int U>
__device__ __forceinline__ int block_append_multi(const bool (&take)[U], const double (&val)[U],
                                                  double* list, int base,
                                                  int (*wsum)[SSN_WAVES_PER_BLOCK]) {
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    unsigned long long m[U];
    int before[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        m[u] = __ballot(take[u]);
        before[u] = __popcll(m[u] & ((1ull << lane) - 1ull));
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int u = 0; u < U; ++u) wsum[u][w] = __popcll(m[u]);
    }
    __syncthreads();
    int off = base;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        int ou = 0, tu = 0;
#pragma unroll
        for (int k = 0; k < SSN_WAVES_PER_BLOCK; ++k) {
            const int c = wsum[u][k];
            if (k < w) ou += c;
            tu += c;
        }
        if (take[u]) list[off + ou + before[u]] = val[u];
        off += tu;
    }
    return off - base;
}

// A 16-byte piece of a row kept raw in registers and widened to fp64 at use.
template <typename T, int VEC> struct RawPiece;
template <> struct RawPiece<double, 2> {
    uint4 u;
    __device__ __forceinline__ double get(int e) const {
        return e == 0 ? __hiloint2double((int)u.y, (int)u.x) : __hiloint2double((int)u.w, (int)u.z);
    }
};
template <> struct RawPiece<float, 4> {
    uint4 u;
    __device__ __forceinline__ double get(int e) const {
        const uint32_t w = e == 0 ? u.x : (e == 1 ? u.y : (e == 2 ? u.z : u.w));
        return (double)__uint_as_float(w);
    }
};
template <> struct RawPiece<bf16_t, 8> {
    uint4 u;
    __device__ __forceinline__ double get(int e) const {
        const uint32_t w = (e >> 1) == 0 ? u.x : ((e >> 1) == 1 ? u.y : ((e >> 1) == 2 ? u.z : u.w));
        return (double)__uint_as_float((e & 1) ? (w & 0xffff0000u) : (w << 16));
    }
};

__device__ __forceinline__ float bf16_to_f32(bf16_t b) {
    return __uint_as_float(((uint32_t)b) << 16);
}

// Element widening to double.
__device__ __forceinline__ double to_f64(double v) { return v; }
__device__ __forceinline__ double to_f64(float v) { return (double)v; }
__device__ __forceinline__ double to_f64(bf16_t v) { return (double)bf16_to_f32(v); }

// Vector load of VEC consecutive elements (16-byte aligned when VEC*sizeof(T) == 16).
template <typename T, int VEC>
struct VecLoad;

template <> struct VecLoad<double, 2> {
    __device__ __forceinline__ static void load(const double* p, double* o) {
        double2 v = *reinterpret_cast<const double2*>(p);
        o[0] = v.x; o[1] = v.y;
    }
};
template <> struct VecLoad<float, 4> {
    __device__ __forceinline__ static void load(const float* p, double* o) {
        float4 v = *reinterpret_cast<const float4*>(p);
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    }
};
template <> struct VecLoad<bf16_t, 8> {
    __device__ __forceinline__ static void load(const bf16_t* p, double* o) {
        uint4 v = *reinterpret_cast<const uint4*>(p);
        uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o[2 * i] = (double)__uint_as_float(w[i] << 16);
            o[2 * i + 1] = (double)__uint_as_float(w[i] & 0xffff0000u);
        }
    }
};
template <typename T> struct VecLoad<T, 1> {
    __device__ __forceinline__ static void load(const T* p, double* o) { o[0] = to_f64(*p); }
};

__device__ __forceinline__ double clampd(double t, double lo, double hi) {
    return fmin(fmax(t, lo), hi);
}

// Appends `val` from every thread with `take` to list[base ...], in thread
// order (deterministic), and returns how many the block appended.  Every
// thread of the block must call it; wsum: SSN_WAVES_PER_BLOCK ints of LDS.
__device__ __forceinline__ int block_append(bool take, double val, double* list, int base,
                                            int* wsum) {
    const int lane = threadIdx.x & (SSN_WAVE - 1), w = threadIdx.x / SSN_WAVE;
    const unsigned long long m = __ballot(take);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    __syncthreads();
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < SSN_WAVES_PER_BLOCK; ++k) {
        if (k < w) off += wsum[k];
        tot += wsum[k];
    }
    if (take) list[base + off + before] = val;
    return tot;
}
