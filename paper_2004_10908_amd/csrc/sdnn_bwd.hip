// Backward kernels of the layered sparse DNN for gfx950.
//
// Chain rule through one layer y_{l+1} = min(c, max(0, y_l W + b)), with the
// derivative of the clipped ReLU taken as 1 on 0 < y_{l+1} < c and 0 elsewhere:
//   G        = dY_{l+1} * [0 < Y_{l+1} < c]
//   db[j]    = sum_r G[r][j]
//   dW[j][k] = sum_r G[r][j] * Y_l[r][idx[j][k]]         (values on the fixed pattern)
//   dY_l[r][i] = sum_{(j,k): idx[j][k] = i} G[r][j] * w[j][k]
// All buffers here are compact: row r of every [R][N] matrix is the r-th row of
// the backward row set, and R is read from device memory.  Every sum has a fixed
// order (no floating-point atomics), so results are bitwise reproducible:
//   dW/db: rows are split into P consecutive groups; a workgroup sums its group's
//          rows in ascending order, a second kernel adds the P partials in order;
//   dY:    the transposed pattern lists each input neuron's (j, k) edges in
//          ascending j*K+k order.
#include "sdnn_internal.hpp"

namespace sdnn {

constexpr int BT = 8;       // rows per tile
constexpr int BNT = 256;    // threads per workgroup

__device__ __forceinline__ float relu_clip_mask(float y, float c) { return (y > 0.f && y < c) ? 1.f : 0.f; }

// dW / db partials.  grid = (P row groups) x (ceil(N / BNT) neuron blocks).
// Each lane owns one neuron and keeps its 32 slot sums; the group's Y_l rows are
// staged BT at a time in LDS, interleaved [N][BT].
__global__ __launch_bounds__(BNT) void k_bwd_dw(BwdDwArgs a) {
    extern __shared__ __align__(16) float lds[];
    const int N = a.N;
    const int R = *a.nrows;
    const int g = blockIdx.x;
    const int r_begin = (int)((int64_t)R * g / a.P);
    const int r_end = (int)((int64_t)R * (g + 1) / a.P);
    const int j = blockIdx.y * BNT + threadIdx.x;
    const bool own = j < N;
    float acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.f;
    float accb = 0.f;
    int ids[K];
    if (own) {
        const int4* ip = reinterpret_cast<const int4*>(a.idx + (size_t)j * K);
#pragma unroll
        for (int q = 0; q < K / 4; ++q) {
            const int4 v = ip[q];
            ids[4 * q] = v.x; ids[4 * q + 1] = v.y; ids[4 * q + 2] = v.z; ids[4 * q + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) ids[k] = 0;
    }
    for (int r0 = r_begin; r0 < r_end; r0 += BT) {
        const int nr = min(BT, r_end - r0);
        __syncthreads();
        for (int e = threadIdx.x; e < BT * N; e += BNT) {
            const int t = e % BT;
            const int i = e / BT;
            lds[e] = t < nr ? a.y_in[(size_t)(r0 + t) * N + i] : 0.f;
        }
        __syncthreads();
        if (own) {
            float gv[BT];
#pragma unroll
            for (int t = 0; t < BT; ++t) {
                if (t < nr) {
                    const size_t o = (size_t)(r0 + t) * N + j;
                    gv[t] = a.dy[o] * relu_clip_mask(a.y_out[o], a.clamp);
                } else {
                    gv[t] = 0.f;
                }
                accb += gv[t];
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float4* p = reinterpret_cast<const float4*>(lds + ids[k] * BT);
                const float4 v0 = p[0], v1 = p[1];
                float s = acc[k];
                s = fmaf(gv[0], v0.x, s); s = fmaf(gv[1], v0.y, s); s = fmaf(gv[2], v0.z, s); s = fmaf(gv[3], v0.w, s);
                s = fmaf(gv[4], v1.x, s); s = fmaf(gv[5], v1.y, s); s = fmaf(gv[6], v1.z, s); s = fmaf(gv[7], v1.w, s);
                acc[k] = s;
            }
        }
    }
    if (own) {
        float4* o = reinterpret_cast<float4*>(a.pdw + ((size_t)g * N + j) * K);
#pragma unroll
        for (int q = 0; q < K / 4; ++q) o[q] = make_float4(acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]);
        a.pdb[(size_t)g * N + j] = accb;
    }
}

// dY_l through the transposed pattern.  Grid-stride over tiles of BT rows; the
// masked gradient G of the tile is staged in LDS, interleaved [N][BT]; each lane
// owns one input neuron and walks its incoming edges.
__global__ __launch_bounds__(BNT) void k_bwd_dy(BwdDyArgs a) {
    extern __shared__ __align__(16) float lds[];
    const int N = a.N;
    const int R = *a.nrows;
    const int ntiles = (R + BT - 1) / BT;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int r0 = tile * BT;
        const int nr = min(BT, R - r0);
        __syncthreads();
        for (int e = threadIdx.x; e < BT * N; e += BNT) {
            const int t = e % BT;
            const int j = e / BT;
            float gval = 0.f;
            if (t < nr) {
                const size_t o = (size_t)(r0 + t) * N + j;
                gval = a.dy[o] * relu_clip_mask(a.y_out[o], a.clamp);
            }
            lds[e] = gval;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < N; i += BNT) {
            float acc[BT];
#pragma unroll
            for (int t = 0; t < BT; ++t) acc[t] = 0.f;
            const int e0 = a.tr_ptr[i], e1 = a.tr_ptr[i + 1];
            for (int p = e0; p < e1; ++p) {
                const int e = a.tr_e[p];
                const float wv = a.w[e];
                const float4* q = reinterpret_cast<const float4*>(lds + (e / K) * BT);
                const float4 v0 = q[0], v1 = q[1];
                acc[0] = fmaf(wv, v0.x, acc[0]); acc[1] = fmaf(wv, v0.y, acc[1]);
                acc[2] = fmaf(wv, v0.z, acc[2]); acc[3] = fmaf(wv, v0.w, acc[3]);
                acc[4] = fmaf(wv, v1.x, acc[4]); acc[5] = fmaf(wv, v1.y, acc[5]);
                acc[6] = fmaf(wv, v1.z, acc[6]); acc[7] = fmaf(wv, v1.w, acc[7]);
            }
#pragma unroll
            for (int t = 0; t < BT; ++t) {
                if (t < nr) {
                    const int r = a.rows_out ? a.rows_out[r0 + t] : r0 + t;
                    a.dy_in[(size_t)r * N + i] = acc[t];
                }
            }
        }
    }
}

int bwd_T() { return BT; }
int bwd_threads() { return BNT; }
const void* bwd_dw_fn() { return (const void*)&k_bwd_dw; }
const void* bwd_dy_fn() { return (const void*)&k_bwd_dy; }

// sum_{g < P} p[g * stride] in g order, with up to 16 loads in flight (a loop that
// adds each value as it arrives waits out one memory latency per partial)
__device__ inline float sum_partials(const float* p, int P, size_t stride) {
    constexpr int U = 16;
    float s = 0.f;
    int g = 0;
    for (; g + U <= P; g += U) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = p[(size_t)(g + u) * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u];
    }
    for (; g < P; ++g) s += p[(size_t)g * stride];
    return s;
}

// dW[j][k] = sum_{g < P} pdw[g][j][k] (in g order); db likewise.
__global__ void k_reduce_partials(const float* pdw, const float* pdb, int32_t P, int32_t N, float* dw, float* db,
                                  const int32_t* nrows, int32_t T) {
    // with a row count: only the first ceil(R / T) partials were written (partial g
    // holds tile stream g, and a stream past the tile count has no tile); R = 0 gives
    // zero gradients
    if (nrows) P = min(P, (*nrows + T - 1) / T);
    const int64_t nk = (int64_t)N * K;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nk + N; e += (int64_t)gridDim.x * blockDim.x) {
        if (e < nk)
            dw[e] = sum_partials(pdw + e, P, (size_t)nk);
        else
            db[e - nk] = sum_partials(pdb + (e - nk), P, (size_t)N);
    }
}

// dst[i][:] = src[rows[i]][:] for i < *n.
__global__ void k_gather_rows(const float* src, const int32_t* rows, const int32_t* n, int32_t N, float* dst) {
    const int R = *n;
    for (int i = blockIdx.x; i < R; i += gridDim.x) {
        const float* s = src + (size_t)rows[i] * N;
        float* d = dst + (size_t)i * N;
        for (int c = threadIdx.x; c < N; c += blockDim.x) d[c] = s[c];
    }
}

// ---------------------------------------------------------------- transposed pattern
__global__ void k_tr_count(const int32_t* idx, int64_t nnz, int32_t* deg) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&deg[idx[e]], 1);
}

// ptr[0..N] = exclusive scan of deg (one workgroup of 1024 threads).
__global__ __launch_bounds__(1024) void k_tr_scan(const int32_t* deg, int32_t N, int32_t* ptr) {
    __shared__ int32_t s[1024];
    const int tid = threadIdx.x;
    const int seg = (N + 1023) / 1024;
    const int i0 = min(N, tid * seg), i1 = min(N, i0 + seg);
    int c = 0;
    for (int i = i0; i < i1; ++i) c += deg[i];
    s[tid] = c;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = tid >= off ? s[tid - off] : 0;
        __syncthreads();
        s[tid] += v;
        __syncthreads();
    }
    int pos = s[tid] - c;
    for (int i = i0; i < i1; ++i) {
        ptr[i] = pos;
        pos += deg[i];
    }
    if (tid == 1023) ptr[N] = s[1023];
}

__global__ void k_tr_fill(const int32_t* idx, int64_t nnz, const int32_t* ptr, int32_t* cursor, int32_t* tr_e) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = idx[e];
        const int pos = ptr[i] + atomicAdd(&cursor[i], 1);
        tr_e[pos] = (int32_t)e;
    }
}

// Sort each input neuron's edge list ascending (insertion sort; lists are ~K long).
__global__ void k_tr_sort(const int32_t* ptr, int32_t N, int32_t* tr_e) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const int a = ptr[i], b = ptr[i + 1];
        for (int p = a + 1; p < b; ++p) {
            const int v = tr_e[p];
            int q = p - 1;
            while (q >= a && tr_e[q] > v) {
                tr_e[q + 1] = tr_e[q];
                --q;
            }
            tr_e[q + 1] = v;
        }
    }
}

}  // namespace sdnn
