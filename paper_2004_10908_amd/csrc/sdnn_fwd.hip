// Forward kernels of the layered sparse DNN for gfx950.
//
// One layer (paper, section "Large Sparse Neural Network Inference"; the layer
// rule of the challenge it runs):  y_{l+1}[r][j] = min(c, max(0, sum_k w[j][k] *
// y_l[r][idx[j][k]] + b[j])) for every alive row r and neuron j.
//
// Work decomposition: a workgroup owns a tile of T activation rows and computes
// all N outputs of those rows, so it alone decides whether each row is still
// alive (has a nonzero) after the layer.  The T input rows are staged in LDS in
// an interleaved [N][T] layout: the T values a neuron needs for one input id are
// contiguous, so one gather is a single 16-byte (or 8/4-byte) LDS read serving T
// rows.  Each lane owns one output neuron at a time, reads its 32 (id, weight)
// pairs with 16-byte global loads and keeps T fp32 accumulators.  The sum runs
// over the slots in ascending order with fused multiply-adds, then adds the bias.
//
// Compaction: rows that come out all-zero are dropped from the next layer's work
// list (an all-zero row stays all-zero while every bias is <= 0).  A workgroup
// ORs per-lane row bits with cross-lane shuffles, reserves list slots with one
// atomic per tile and appends its alive rows.  Row values never move; only the
// list of row ids shrinks.  The order of the list depends on atomic order, but a
// row's arithmetic does not depend on its position, so outputs are bitwise
// deterministic.  Once a layer's list is empty every later layer returns at once
// (early exit), the GPU counterpart of the paper's condition-task loop that
// stops dispatching.
#include "sdnn_internal.hpp"
#include "sdnn_device.hpp"

namespace sdnn {

template <int T>
__device__ __forceinline__ void gather_fma(const float* __restrict__ lds, int i, float w, float (&acc)[T]) {
    const float* p = lds + i * T;
    if constexpr (T == 1) {
        acc[0] = fmaf(w, p[0], acc[0]);
    } else if constexpr (T == 2) {
        const float2 v = *reinterpret_cast<const float2*>(p);
        acc[0] = fmaf(w, v.x, acc[0]);
        acc[1] = fmaf(w, v.y, acc[1]);
    } else {
#pragma unroll
        for (int h = 0; h < T / 4; ++h) {
            const float4 v = reinterpret_cast<const float4*>(p)[h];
            acc[4 * h + 0] = fmaf(w, v.x, acc[4 * h + 0]);
            acc[4 * h + 1] = fmaf(w, v.y, acc[4 * h + 1]);
            acc[4 * h + 2] = fmaf(w, v.z, acc[4 * h + 2]);
            acc[4 * h + 3] = fmaf(w, v.w, acc[4 * h + 3]);
        }
    }
}

// Direct variant: the T rows are read from global memory (rows too wide for LDS).
template <int T>
__device__ __forceinline__ void gather_fma_direct(const float* const (&yr)[T], int i, float w, float (&acc)[T]) {
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = fmaf(w, yr[t][i], acc[t]);
}

// Unroll of the slot loop (4 slots per step): enough independent LDS reads in
// flight to cover latency without exceeding the VGPR budget of NT threads per CU.
template <int T, int NT>
constexpr int slot_unroll() {
    constexpr int budget = NT <= 256 ? 200 : (NT <= 512 ? 160 : 96);
    constexpr int per_step = 8 + 4 * T;
    constexpr int u = (budget - 3 * T) / per_step;
    return u < 1 ? 1 : (u > 8 ? 8 : u);
}

// All tiles of one layer handled by workgroup `wg` of `nwg` (grid-stride).
template <int T, int NT, bool STAGED>
__device__ __forceinline__ void run_layer(const LayerArgs& a, float* __restrict__ lds, int wg, int nwg, int R) {
    __shared__ int32_t s_rows[T];
    __shared__ unsigned s_alive;
    constexpr int UQ = slot_unroll<T, NT>();
    const int N = a.N;
    const int tid = threadIdx.x;
    const int ntiles = (R + T - 1) / T;
    for (int tile = wg; tile < ntiles; tile += nwg) {
        if (tid < T) {
            const int p = tile * T + tid;
            s_rows[tid] = p < R ? (a.list_in ? a.list_in[p] : a.row_base + p) : -1;
        }
        if (tid == 0) s_alive = 0u;
        __syncthreads();
        int rr[T];
#pragma unroll
        for (int t = 0; t < T; ++t) rr[t] = s_rows[t];
        if constexpr (STAGED) {
            // interleaved [N][T] staging: consecutive threads fill consecutive LDS words
            for (int e = tid; e < T * N; e += NT) {
                const int t = e % T;
                const int i = e / T;
                const int r = s_rows[t];
                lds[e] = r >= 0 ? a.yin[(size_t)r * N + i] : 0.f;
            }
            __syncthreads();
        }
        const float* yr[T];
#pragma unroll
        for (int t = 0; t < T; ++t) yr[t] = a.yin + (size_t)(rr[t] >= 0 ? rr[t] : 0) * N;
        unsigned bits = 0u;
        for (int j = tid; j < N; j += NT) {
            float acc[T];
#pragma unroll
            for (int t = 0; t < T; ++t) acc[t] = 0.f;
            const int4* ip = reinterpret_cast<const int4*>(a.idx + (size_t)j * K);
            const float4* wp = reinterpret_cast<const float4*>(a.w + (size_t)j * K);
#pragma unroll UQ
            for (int q = 0; q < K / 4; ++q) {
                const int4 iv = ip[q];
                const float4 wv = wp[q];
                if constexpr (STAGED) {
                    gather_fma<T>(lds, iv.x, wv.x, acc);
                    gather_fma<T>(lds, iv.y, wv.y, acc);
                    gather_fma<T>(lds, iv.z, wv.z, acc);
                    gather_fma<T>(lds, iv.w, wv.w, acc);
                } else {
                    gather_fma_direct<T>(yr, iv.x, wv.x, acc);
                    gather_fma_direct<T>(yr, iv.y, wv.y, acc);
                    gather_fma_direct<T>(yr, iv.z, wv.z, acc);
                    gather_fma_direct<T>(yr, iv.w, wv.w, acc);
                }
            }
            const float bj = a.b[j];
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const float y = fminf(fmaxf(acc[t] + bj, 0.f), a.clamp);
                if (rr[t] >= 0) {
                    const size_t o = (size_t)rr[t] * N + j;
                    a.yout[o] = y;
                    if (a.ycopy) a.ycopy[o] = y;
                }
                bits |= (y != 0.f ? 1u : 0u) << t;
            }
        }
        // row liveness: OR over every neuron of the tile
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) bits |= __shfl_xor(bits, off);
        if ((tid & 63) == 0 && bits) atomicOr(&s_alive, bits);
        __syncthreads();
        const unsigned alive = s_alive;
        if (tid == 0 && a.list_out) {
            int n = 0;
#pragma unroll
            for (int t = 0; t < T; ++t) n += (rr[t] >= 0 && ((alive >> t) & 1u)) ? 1 : 0;
            if (n) {
                int base = atomicAdd(a.cnt_out, n);
#pragma unroll
                for (int t = 0; t < T; ++t)
                    if (rr[t] >= 0 && ((alive >> t) & 1u)) a.list_out[base++] = rr[t];
            }
        }
        if (a.alive && tid < T) {
            const int r = s_rows[tid];
            if (r >= 0) a.alive[r] = ((alive >> tid) & 1u) ? 1 : a.dead_mark;
        }
        __syncthreads();
    }
}

template <int T, int NT, bool STAGED>
__global__ __launch_bounds__(NT) void k_layer(LayerArgs a) {
    extern __shared__ __align__(16) float lds[];
    const int R = a.cnt_in ? *a.cnt_in : a.nrows;
    run_layer<T, NT, STAGED>(a, lds, blockIdx.x, gridDim.x, R);
}

// ---------------------------------------------------------------- finalize
// Ascending ids of rows whose final activations are nonzero, and the per-layer
// row profile.  Two passes of FIN_BLOCKS workgroups over consecutive row ranges:
// k_fin_count counts each range's alive rows (coalesced loads); k_fin_write gives
// each range its output offset (the sum of the ranges before it) and writes its
// rows in ascending order, 1024 at a time, each wave placing its rows with a
// ballot and the waves in order through LDS.
constexpr int FIN_NT = 1024;

__device__ __forceinline__ void fin_range(int32_t rows, int64_t* r0, int64_t* r1) {
    const int64_t per = ((int64_t)rows + FIN_BLOCKS - 1) / FIN_BLOCKS;
    *r0 = min((int64_t)rows, (int64_t)blockIdx.x * per);
    *r1 = min((int64_t)rows, *r0 + per);
}

__global__ __launch_bounds__(FIN_NT) void k_fin_count(const int32_t* alive, int32_t rows, int32_t* part) {
    __shared__ int s_w[FIN_NT / 64];
    int64_t r0, r1;
    fin_range(rows, &r0, &r1);
    int c = 0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += FIN_NT) c += alive[r] > 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < FIN_NT / 64; ++w) t += s_w[w];
        part[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(FIN_NT) void k_fin_write(const int32_t* alive, int32_t rows, const int32_t* part,
                                                      int32_t* nz_rows, int32_t* n_nz, const int32_t* cnt,
                                                      int32_t n_regions, int32_t L, int32_t* layer_rows,
                                                      const int32_t* err, int32_t* host_err) {
    __shared__ int s_w[FIN_NT / 64];
    __shared__ int s_base;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int64_t r0, r1;
    fin_range(rows, &r0, &r1);
    if (tid == 0) {
        int b = 0;
        for (int i = 0; i < (int)blockIdx.x; ++i) b += part[i];
        s_base = b;
        if (blockIdx.x == 0) {
            int total = 0;
            for (int i = 0; i < FIN_BLOCKS; ++i) total += part[i];
            *n_nz = total;
            if (layer_rows) layer_rows[L] = total;
            // a device error raised by this forward (or injected) becomes visible to the
            // host without a synchronization: the library's next call reports it
            const int32_t e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (e != 0 && host_err) __hip_atomic_store(host_err, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
    if (blockIdx.x == 0 && layer_rows) {
        for (int l = tid; l < L; l += FIN_NT) {
            int sum = 0;
            for (int g = 0; g < n_regions; ++g) sum += cnt[(size_t)g * (L + 1) + l];
            layer_rows[l] = sum;
        }
    }
    __syncthreads();
    int base = s_base;
    for (int64_t rc = r0; rc < r1; rc += FIN_NT) {
        const int64_t r = rc + tid;
        const bool f = r < r1 && alive[r] > 0;
        const unsigned long long m = __ballot(f);
        if (lane == 0) s_w[wave] = __popcll(m);
        __syncthreads();
        int woff = 0, tot = 0;
        for (int w = 0; w < FIN_NT / 64; ++w) {
            woff += w < wave ? s_w[w] : 0;
            tot += s_w[w];
        }
        if (f) nz_rows[base + woff + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)r;
        base += tot;
        __syncthreads();                           // s_w is rewritten next round
    }
}

// Rows whose alive flag is -1 died in a layer that wrote the other ping-pong
// buffer, so the output buffer still holds their older values: clear them (one
// workgroup per row at a time, 16-byte stores; N is a multiple of 4 or the tail is
// written by 4-byte stores).
__global__ __launch_bounds__(256) void k_fin_zero(const int32_t* alive, int32_t rows, int32_t N, float* y_out) {
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        if (alive[r] >= 0) continue;                 // uniform over the workgroup
        float* y = y_out + (size_t)r * N;
        if ((N & 3) == 0) {
            float4* y4 = reinterpret_cast<float4*>(y);
            for (int i = threadIdx.x; i < N / 4; i += 256) y4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
            for (int i = threadIdx.x; i < N; i += 256) y[i] = 0.f;
        }
    }
}

// ---------------------------------------------------------------- persistent chain
// All layers in one cooperative launch: layer l's tiles are spread over the
// co-resident grid, a grid barrier separates layers, and the loop stops as soon
// as a layer's work list is empty.  Layer l writes X_l, which is y_out when
// (L-1-l) is even and the workspace buffer otherwise, so the last layer always
// lands in y_out.
template <int T, int NT, bool STAGED>
__global__ __launch_bounds__(NT) void k_chain(ChainArgs) {
    extern __shared__ __align__(16) float lds[];
    __shared__ int s_ok;
    unsigned gen = 0u;
    for (int l = 0;; ++l) {
        {
            const ChainArgs c = reload_chain_args();
            if (l >= c.L) break;
            const int R = (l == 0 || !c.compaction) ? c.rows : ld_count(&c.cnt[l]);
            if (R == 0) break;
            const LayerArgs a = chain_layer_args(c, l, R);
            run_layer<T, NT, STAGED>(a, lds, blockIdx.x, gridDim.x, R);
        }
        const ChainArgs c = reload_chain_args();
        if (!grid_barrier(c.bar, gen, c.err, &s_ok)) return;
    }
    // the nz list and the row profile are produced by the finalize passes after this kernel
}

// ---------------------------------------------------------------- wide-layer kernels
// For layers too wide for a tile of several rows in LDS (by default where not even
// 2 rows fit, e.g. 65536 neurons), a layer is two passes:
//  * pack: the rows of the work list, T at a time, are copied into a workspace
//    buffer as tiles [tile][N][T], so the T values of one input id are contiguous;
//  * compute: a gather of input id i is then T * 4 contiguous bytes serving T rows,
//    instead of T scattered 4-byte loads; the T / 4 lanes of a neuron take 16 bytes
//    (4 rows) each, so one load instruction reads whole slots.  Tile X goes to
//    workgroup group X % 8 (group = blockIdx % 8, the XCD it runs on); the
//    workgroups of a group split each of its tiles by chunks of 4 NT / T neurons
//    (their 32 (id, weight) pairs read per tile), so the gathers from a tile all
//    go through one XCD's L2 (a tile larger than the L2, 32 rows of 65536 floats,
//    is served from the Infinity Cache).  A group with at least twice as many
//    workgroups as chunks runs several tile sub-streams.
//    The last workgroup to finish a tile (a counter per tile) publishes its row
//    liveness: list slots, alive flags, dead rows zeroed where asked.
// The per-output arithmetic is run_layer's (slots in ascending order with fused
// multiply-adds, then the bias), so outputs are bitwise equal to it.

template <int T>
__device__ __forceinline__ void wide_pack_body(const LayerArgs& a, int R, int wg, int nwg) {
    __shared__ int32_t s_prow[T];
    const int N = a.N;
    const int nt = blockDim.x;
    const int64_t ntiles = (R + T - 1) / T;
    const int chunk = 4 * nt;                              // ids per task
    const int64_t chunks = (N + chunk - 1) / chunk;
    for (int64_t task = wg; task < ntiles * chunks; task += nwg) {
        const int64_t tile = task / chunks;
        const int c0 = (int)(task % chunks) * chunk;
        __syncthreads();                                   // the previous task's row ids are read
        if ((int)threadIdx.x < T) {
            const int64_t p = tile * T + threadIdx.x;
            s_prow[threadIdx.x] = p < R ? (a.list_in ? a.list_in[p] : a.row_base + (int32_t)p) : -1;
        }
        __syncthreads();
        int32_t rr[T];
#pragma unroll
        for (int t = 0; t < T; ++t) rr[t] = s_prow[t];
        float* dst = a.packed + (size_t)tile * N * T;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = c0 + q * nt + (int)threadIdx.x;
            if (i < N) {
                float v[T];
#pragma unroll
                for (int t = 0; t < T; ++t) v[t] = rr[t] >= 0 ? a.yin[(size_t)rr[t] * N + i] : 0.f;
                float4* o = reinterpret_cast<float4*>(dst + (size_t)i * T);
#pragma unroll
                for (int h = 0; h < T / 4; ++h) o[h] = make_float4(v[4 * h], v[4 * h + 1], v[4 * h + 2], v[4 * h + 3]);
            }
        }
    }
}

template <int T>
__global__ __launch_bounds__(WIDE_PACK_NT) void k_wide_pack(LayerArgs a) {
    const int R = a.cnt_in ? *a.cnt_in : a.nrows;
    wide_pack_body<T>(a, R, blockIdx.x, gridDim.x);
}

// slot groups (4 slots each) whose gathers the compiler may keep in flight together.
// Layer kernel at 1024 threads: one group (56 VGPRs) lets two workgroups share a CU,
// which beat four groups with one workgroup per CU (C4 layer 15.2 against 15.9 ms);
// at 512 threads four groups are faster (20.3 against 26.6 ms).  The persistent chain
// holds one 1024-thread workgroup per CU either way (its pack and barrier code need
// more registers), so it keeps four groups (C4 forward 29.0 against 33.2 ms).
template <int NT, bool CHAIN>
constexpr int wide_unroll() { return (NT >= 1024 && !CHAIN) ? 1 : 4; }

// The Q = T / 4 lanes of one neuron split the tile's rows, 4 each: lane quarter rq
// reads bytes 16 rq .. 16 rq + 15 of the T * 4-byte slot, so one load instruction
// fetches 64 / Q whole slots (contiguous segments) rather than 64 scattered pieces.
template <int T, int NT, int UNROLL>
__device__ __forceinline__ void run_layer_wide(const LayerArgs& a, int wg, int nwg, int R) {
    static_assert(T % 4 == 0 && T <= 32, "T rows must fit the 32 row bits of a tile word");
    constexpr int Q = T / 4;                       // lanes per neuron
    constexpr int NPC = NT / Q;                    // neurons per chunk
    static_assert(64 % Q == 0 && NT % 64 == 0, "a neuron's lanes must sit in one wave");
    __shared__ int32_t s_rows[T];
    __shared__ unsigned s_bits;
    __shared__ int s_last;
    const int N = a.N;
    const int tid = threadIdx.x;
    const int rq = tid % Q;                        // rows 4 rq .. 4 rq + 3 of the tile
    const int jl = tid / Q;                        // neuron within the chunk
    const int ntiles = (R + T - 1) / T;
    const int groups = nwg < 8 ? nwg : 8;
    const int grp = wg & 7;                        // < groups: wg < nwg
    const int gi = wg >> 3;                        // index within the group
    const int gsize = (nwg - grp + 7) >> 3;        // workgroups of the group
    const int nch = (N + NPC - 1) / NPC;           // neuron chunks
    const int per = gsize < nch ? gsize : nch;     // workgroups sharing one tile
    const int sub = gsize / per;                   // tile sub-streams of the group
    const int s = gi / per, ci = gi % per;
    if (s >= sub) return;                          // no share of any tile
    for (int tile = grp + groups * s; tile < ntiles; tile += groups * sub) {
        if (tid < T) {
            const int p = tile * T + tid;
            s_rows[tid] = p < R ? (a.list_in ? a.list_in[p] : a.row_base + p) : -1;
        }
        if (tid == 0) s_bits = 0u;
        __syncthreads();
        // rows past the list end sit at the tile's end
        const int nvalid = R - tile * T < T ? R - tile * T : T;
        const unsigned valid = nvalid >= 32 ? ~0u : ((1u << nvalid) - 1u);
        const float4* tq = reinterpret_cast<const float4*>(a.packed + (size_t)tile * N * T) + rq;
        unsigned bits = 0u;
        for (int c = ci; c < nch; c += per) {
            const int j = c * NPC + jl;
            if (j < N) {
                float acc[4] = {0.f, 0.f, 0.f, 0.f};
                auto slot = [&](int i, float w) {
                    const float4 v = tq[(size_t)i * Q];
                    acc[0] = fmaf(w, v.x, acc[0]);
                    acc[1] = fmaf(w, v.y, acc[1]);
                    acc[2] = fmaf(w, v.z, acc[2]);
                    acc[3] = fmaf(w, v.w, acc[3]);
                };
                const int4* ip = reinterpret_cast<const int4*>(a.idx + (size_t)j * K);
                const float4* wp = reinterpret_cast<const float4*>(a.w + (size_t)j * K);
#pragma unroll UNROLL
                for (int q = 0; q < K / 4; ++q) {
                    const int4 iv = ip[q];
                    const float4 wv = wp[q];
                    slot(iv.x, wv.x);
                    slot(iv.y, wv.y);
                    slot(iv.z, wv.z);
                    slot(iv.w, wv.w);
                }
                const float bj = a.b[j];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int row = 4 * rq + t;
                    const float y = fminf(fmaxf(acc[t] + bj, 0.f), a.clamp);
                    if (row < nvalid) {
                        const size_t o = (size_t)s_rows[row] * N + j;
                        a.yout[o] = y;
                        if (a.ycopy) a.ycopy[o] = y;
                    }
                    bits |= (y != 0.f ? 1u : 0u) << row;
                }
            }
        }
        bits &= valid;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) bits |= __shfl_xor(bits, off);
        if ((tid & 63) == 0 && bits) atomicOr(&s_bits, bits);
        __syncthreads();
        if (tid == 0) {
            int32_t* wd = a.wide_words + 2 * (size_t)tile;
            const unsigned mine = s_bits;
            __threadfence();
            if (mine) atomicOr(reinterpret_cast<unsigned*>(wd), mine);
            __threadfence();
            const int last = atomicAdd(wd + 1, 1) == per - 1;
            if (last) {
                __threadfence();
                s_bits = (unsigned)__hip_atomic_load(wd, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                atomicExch(wd, 0);                 // every sharer has arrived: reset for the next layer
                atomicExch(wd + 1, 0);
            }
            s_last = last;
        }
        __syncthreads();
        if (s_last) {
            const unsigned alive = s_bits;
            if (tid == 0 && a.list_out) {
                const int n = __popc(alive);
                if (n) {
                    int base = atomicAdd(a.cnt_out, n);
#pragma unroll
                    for (int t = 0; t < T; ++t)
                        if ((alive >> t) & 1u) a.list_out[base++] = s_rows[t];
                }
            }
            if (a.alive && tid < nvalid) a.alive[s_rows[tid]] = ((alive >> tid) & 1u) ? 1 : a.dead_mark;
        }
        __syncthreads();                           // s_rows, s_bits, s_last are reused
    }
}

template <int T, int NT>
__global__ __launch_bounds__(NT) void k_layer_wide(LayerArgs a) {
    const int R = a.cnt_in ? *a.cnt_in : a.nrows;
    run_layer_wide<T, NT, wide_unroll<NT, false>()>(a, blockIdx.x, gridDim.x, R);
}

// Persistent chain of the wide kernels: pack, grid barrier, compute, grid barrier.
template <int T, int NT>
__global__ __launch_bounds__(NT) void k_chain_wide(ChainArgs) {
    __shared__ int s_ok;
    unsigned gen = 0u;
    for (int l = 0;; ++l) {
        int R;
        {
            const ChainArgs c = reload_chain_args();
            if (l >= c.L) break;
            R = (l == 0 || !c.compaction) ? c.rows : ld_count(&c.cnt[l]);
            if (R == 0) break;
            const LayerArgs a = chain_layer_args(c, l, R);
            wide_pack_body<T>(a, R, blockIdx.x, gridDim.x);
            if (!grid_barrier(c.bar, gen, c.err, &s_ok)) return;
        }
        {
            // run_layer_wide returns early only in workgroups with no share of any tile,
            // which then wait at the barrier below like the others
            const ChainArgs c = reload_chain_args();
            const LayerArgs a = chain_layer_args(c, l, R);
            run_layer_wide<T, NT, wide_unroll<NT, true>()>(a, blockIdx.x, gridDim.x, R);
        }
        const ChainArgs c = reload_chain_args();
        if (!grid_barrier(c.bar, gen, c.err, &s_ok)) return;
    }
}

// 16-byte LDS read at an absolute LDS byte address (the offsets already include
// the workgroup's LDS base), so the address register is used as is.
__device__ __forceinline__ float4 lds_read16(uint32_t addr) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef float v4f __attribute__((ext_vector_type(4)));
    __builtin_assume((addr & 15u) == 0u);
    const v4f r = *reinterpret_cast<const v4f __attribute__((address_space(3)))*>(addr);
    return make_float4(r.x, r.y, r.z, r.w);
#else
    (void)addr;   // host pass of a device-only function
    return make_float4(0.f, 0.f, 0.f, 0.f);
#endif
}

// 4-byte LDS read and 16-byte LDS write at absolute LDS byte addresses.
__device__ __forceinline__ float lds_read4(uint32_t addr) {
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_assume((addr & 3u) == 0u);
    return *reinterpret_cast<const float __attribute__((address_space(3)))*>(addr);
#else
    (void)addr;
    return 0.f;
#endif
}
__device__ __forceinline__ void lds_write16(uint32_t addr, float4 v) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef float v4f __attribute__((ext_vector_type(4)));
    __builtin_assume((addr & 15u) == 0u);
    v4f r = {v.x, v.y, v.z, v.w};
    *reinterpret_cast<v4f __attribute__((address_space(3)))*>(addr) = r;
#else
    (void)addr;
    (void)v;
#endif
}

// 8-byte LDS read at an absolute LDS byte address.
__device__ __forceinline__ uint2 lds_read8(uint32_t addr) {
#if defined(__HIP_DEVICE_COMPILE__)
    typedef unsigned v2u __attribute__((ext_vector_type(2)));
    __builtin_assume((addr & 7u) == 0u);
    const v2u r = *reinterpret_cast<const v2u __attribute__((address_space(3)))*>(addr);
    return make_uint2(r.x, r.y);
#else
    (void)addr;
    return make_uint2(0u, 0u);
#endif
}

// ---------------------------------------------------------------- scheduled kernel
// Resident-weight variant for layers whose 4-row tile fits LDS twice
// (N <= 4096 or so).  A workgroup of 512 lanes owns 1024 neurons ("part") for the
// whole layer: each lane keeps the slot schedule (LDS byte offsets) and weights
// of two neurons in registers, so the weights are read once per layer per
// workgroup instead of once per tile.  The slot order comes from the create-time
// scheduler, so every 16-byte LDS read of a lane unit hits 16 distinct bank
// groups.  With G parts per layer (G = ceil(N / 1024)), the G workgroups that
// share a tile combine their row bits with one device atomic each; the last one
// to finish the tile appends the alive rows, writes the alive flags and zeroes
// dead rows where needed.  Workgroup b serves part (b/8) % G of tile stream
// (b/(8G))*8 + b%8, so the parts of a tile run on the same XCD (blockIdx % 8)
// and share its L2.
//
// LDS: two tile buffers [id][row] (16 bytes per id, the 4 rows of one input: one
// 16-byte read feeds 4 FMAs) in blocks of 64 ids, the blocks of the two buffers
// interleaved: block m of buffer b at byte 2048 m + 1024 b, so an id's offset is
// 2048 (id / 64) + 16 (id % 64) in buffer 0 and the same + an immediate 1024 in
// buffer 1, and its bank group is id mod 16 in either.  Then 128 bytes of scalars,
// the output staging area, the overflow area.
//
// The next tile arrives in the other buffer with asynchronous 16-byte global->LDS
// copies while this one is being read.  A copy lands its 64 lanes' 16 bytes in lane
// order, so one copy of block m brings rows 0..3 of ids 64m .. 64m+63 as [row][id]
// (lane l: row l / 16, ids 64m + 4 (l % 16) .. +3); the wave that issued it turns
// the block into [id][row] in place once it has landed (four 4-byte reads and one
// 16-byte write per lane), before the barrier that hands the tile to the compute.
// 16-byte copies move four times as much per instruction as 4-byte ones, which is
// what bounds the staging rate.
struct SchedLds {
    unsigned* scalars;    // 32 words
    float* out;           // [waves][4][128] each wave's outputs of one tile (its two blocks)
    uint32_t base;        // LDS byte address of the tile buffers
    uint32_t ovf;         // LDS byte address of the overflow area
    int N;
    __device__ __forceinline__ SchedLds(float* lds, int n)
        : scalars(reinterpret_cast<unsigned*>(lds + sched_tile_bytes(n) / 4)),
          out(lds + sched_tile_bytes(n) / 4 + SCHED_SCALARS / 4), base((uint32_t)(uintptr_t)lds),
          ovf((uint32_t)(uintptr_t)lds + (uint32_t)sched_tile_bytes(n) + SCHED_SCALARS + SCHED_OUT), N(n) {}
    // blocks of 64 ids; the last one may be partial (N % 64 ids)
    __device__ __forceinline__ int blocks() const { return (N + 63) >> 6; }
    // blocks a wave copies (and transposes): wave, wave + waves, ...
    __device__ __forceinline__ int blocks_of(int wave, int waves) const {
        const int total = blocks();
        return wave < total ? (total - wave + waves - 1) / waves : 0;
    }
    // the lane's byte offset within a block copy: row `row` (the tile row l / 16),
    // ids 4 (l % 16) .. +3
    __device__ __forceinline__ uint32_t lane_off(int row, int lane) const {
        return 4u * ((uint32_t)row * (uint32_t)N + 4u * (uint32_t)(lane & 15));
    }
    // A wave's copies of one tile as a cursor: blocks m = wave + i * waves, i = 0 ..
    // full-1, then the partial last block (if this wave owns it) with its lanes past
    // N switched off.  Scalar source address (id 64m of row 0) and LDS destination
    // advance by one stride per copy.  The caller guarantees rows * N * 4 < 2^32.
    template <int WAVES>
    struct Cursor {
        uint64_t src;     // global byte address of id 64m of row 0 (the lane's row is in voff)
        uint32_t dst;     // LDS byte address of block m in the target buffer
        uint32_t voff;
        int full;         // full blocks left
        int partial;      // 1: the partial last block after them
        bool lane_in;     // the lane's ids of the partial block are < N
        __device__ __forceinline__ void copy() const {
            uint32_t saved;
            __asm__ volatile(
                "s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\tglobal_load_lds_dwordx4 %1, %3\n\ts_mov_b32 m0, %0"
                : "=&s"(saved) : "v"(voff), "s"(dst), "s"(src) : "memory");
        }
        __device__ __forceinline__ void issue() {
            if (full > 0) {
                copy();
                src += 256u * WAVES;
                dst += 2048u * WAVES;
                --full;
            }
        }
        __device__ __forceinline__ void finish() {
            while (full > 0) issue();
            if (partial) {
                if (lane_in) copy();
                partial = 0;
            }
        }
    };
    template <int WAVES>
    __device__ __forceinline__ Cursor<WAVES> cursor(const float* src, int row, int lane, int wave, int buf,
                                                    bool on) const {
        Cursor<WAVES> k;
        const uint64_t gb = (uint64_t)(uintptr_t)(src + 64 * wave);
        // (readfirstlane returns int: widen through uint32_t, never by sign extension)
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)gb);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(gb >> 32));
        k.src = ((uint64_t)hi << 32) | (uint64_t)lo;
        k.dst = __builtin_amdgcn_readfirstlane(base + 2048u * (uint32_t)wave + 1024u * (uint32_t)buf);
        k.voff = lane_off(row, lane);
        const int n = on ? blocks_of(wave, WAVES) : 0;
        const bool has_partial = (N & 63) && n > 0 && wave + (n - 1) * WAVES == blocks() - 1;
        k.full = has_partial ? n - 1 : n;
        k.partial = has_partial ? 1 : 0;
        k.lane_in = 4 * (lane & 15) < (N & 63);
        return k;
    }
    // The wave's landed blocks of buffer `buf`, [row][id] -> [id][row] in place (the
    // caller has waited for its copies): lane l gathers the 4 rows of id 64m + l and
    // writes them back as one 16-byte slot.  NB blocks at a time: all their reads
    // are issued before any write, and LDS serves a wave's instructions in order.
    // (Slots of ids >= N in a partial block get junk, which nothing reads.)
    template <int WAVES, int NB>
    __device__ __forceinline__ void transpose(int wave, int lane, int buf) const {
        const int n = blocks_of(wave, WAVES);
        const uint32_t r0 = base + 2048u * (uint32_t)wave + 1024u * (uint32_t)buf + 4u * (uint32_t)lane;
        const uint32_t w0 = r0 + 12u * (uint32_t)lane;   // the lane's 16-byte slot in the block
        for (int i0 = 0; i0 < n; i0 += NB) {
            // one uniform test per block; the reads of a present block are straight-line
            float x[NB][4];
            // (addresses as base + a constant below 64 KB, so each read and write
            // takes its offset as an immediate)
            constexpr uint32_t BS = 2048u * WAVES;           // bytes between a wave's blocks
            constexpr int PER = (int)(65536u / BS) > 0 ? (int)(65536u / BS) : 1;   // blocks per base
            const uint32_t rb = r0 + BS * (uint32_t)i0, wb = w0 + BS * (uint32_t)i0;
#pragma unroll
            for (int u = 0; u < NB; ++u)
                if (i0 + u < n) {
                    const uint32_t rbu = rb + BS * (uint32_t)(u / PER * PER);
#pragma unroll
                    for (int r = 0; r < 4; ++r) x[u][r] = lds_read4(rbu + BS * (uint32_t)(u % PER) + 256u * r);
                }
#pragma unroll
            for (int u = 0; u < NB; ++u)
                if (i0 + u < n) {
                    const uint32_t wbu = wb + BS * (uint32_t)(u / PER * PER);
                    lds_write16(wbu + BS * (uint32_t)(u % PER), make_float4(x[u][0], x[u][1], x[u][2], x[u][3]));
                }
        }
    }
};

// Lanes 0..3 of a wave: one dword each from src[lane] into dst[lane] (an LDS
// pointer), asynchronously; waited for with the tile's copies.
__device__ __forceinline__ void lds_copy4(const int32_t* src, int* dst_lds) {
    const uint32_t dst = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)dst_lds);
    uint32_t saved;
    __asm__ volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\tglobal_load_lds_dword %1, off\n\ts_mov_b32 m0, %0"
                     : "=&s"(saved) : "v"(src), "s"(dst) : "memory");
}

// The same for words other workgroups keep changing: a device-scope read (sc1)
// that skips this CU's vector cache.
__device__ __forceinline__ void lds_copy4_coherent(const int32_t* src, int* dst_lds) {
    const uint32_t dst = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)dst_lds);
    uint32_t saved;
    __asm__ volatile("s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\tglobal_load_lds_dword %1, off sc1\n\ts_mov_b32 m0, %0"
                     : "=&s"(saved) : "v"(src), "s"(dst) : "memory");
}

// Loose lockstep of the parts of a tile stream.  The G workgroups that share a
// tile read the same 64 KB from memory; when they run within a few tiles of each
// other, the L2 serves most of those reads, but parts with lighter schedules drift
// ahead (by tens of tiles over a layer).  Each part publishes its tile count;
// a part more than SCHED_AHEAD tiles ahead of its slowest sibling waits for it,
// for at most SCHED_WAIT_TICKS of the 100 MHz clock, and then goes on regardless:
// this is a cache-locality measure only, results never depend on it.
constexpr int SCHED_AHEAD = 2;
constexpr uint64_t SCHED_WAIT_TICKS = 2000;   // 20 us per tile
__device__ __forceinline__ int part_progress(int v, unsigned tag) {
    return ((unsigned)v & 0xfff00000u) == tag ? (int)((unsigned)v & 0xfffffu) : -1;
}


// One lane's resident neuron: schedule offsets and weights of one 64-neuron block.
// Steps past DMAX (rare long blocks) are kept in LDS as (offset, weight) pairs
// when the workgroup's overflow area has room, else read from memory.
template <int DMAX>
struct SchedNeuron {
    uint32_t off[DMAX];
    float wv[DMAX];
    int D, slot, j;
    float bj;
    uint32_t ovf;   // LDS byte address of this block's overflow pairs (64 lanes x 8 bytes per step), or ~0u
    __device__ __forceinline__ float weight_of(const LayerArgs& a, uint32_t e, int st) const {
        const bool pad = (e & 0x80000000u) || j < 0;
        return pad ? 0.f : (a.ent_w ? a.w[a.ent_w[(size_t)st * (a.nblk * 64) + slot]] : a.w[(size_t)j * K + (e & 31u)]);
    }
    // d_even / d_odd: register steps of the part's even / odd blocks (for the
    // overflow area's block order)
    __device__ __forceinline__ void load(const LayerArgs& a, int first_blk, int blk, int lane, uint32_t lds_base,
                                         uint32_t ovf_base, float* lds, int d_even, int d_odd) {
        const bool have = blk < a.nblk;
        slot = blk * 64 + lane;
        j = have ? a.lane_neuron[slot] : -1;
        D = have ? __builtin_amdgcn_readfirstlane(a.wave_steps[blk]) : 0;
        // entries hold the byte offset of the slot's id in the compute tile (16 id) and the slot;
        // all loads are issued before any is waited for
        uint32_t e[DMAX];
#pragma unroll
        for (int st = 0; st < DMAX; ++st)
            e[st] = (have && st < D) ? a.ent[(size_t)st * (a.nblk * 64) + slot] : (0x80000000u | 31u);
#pragma unroll
        for (int st = 0; st < DMAX; ++st) {
            off[st] = lds_base + ((e[st] >> 5) & 0x03ffffffu);
            wv[st] = weight_of(a, e[st], st);
        }
        bj = (j >= 0 && a.b) ? a.b[j] : 0.f;
        ovf = ~0u;
        if (D > DMAX) {
            // the part's blocks take the overflow area in block order
            int pre = 0;
            for (int b2 = first_blk; b2 < blk; ++b2)
                pre += max(0, __builtin_amdgcn_readfirstlane(a.wave_steps[b2]) - (((b2 - first_blk) & 1) ? d_odd : d_even));
            if (pre + (D - DMAX) <= SCHED_OVF) {
                ovf = ovf_base + (uint32_t)pre * 512u;
                uint2* dst = reinterpret_cast<uint2*>(reinterpret_cast<char*>(lds) + (ovf - lds_base)) + lane;
                for (int st = DMAX; st < D; ++st) {
                    const uint32_t x = a.ent[(size_t)st * (a.nblk * 64) + slot];
                    dst[(st - DMAX) * 64] =
                        make_uint2(lds_base + ((x >> 5) & 0x03ffffffu), __float_as_uint(weight_of(a, x, st)));
                }
            }
        }
#pragma unroll
        for (int st = 0; st < DMAX; ++st) __asm__ volatile("" : "+v"(off[st]), "+v"(wv[st]));   // keep resident
    }
};

// An empty asm that takes 16 values as inputs and outputs: the compiler must have
// all of them (one wait for the last) before the asm and cannot move their uses
// above it.
__device__ __forceinline__ void consume16(float4 (&v)[4]) {
    __asm__ volatile(""
                     : "+v"(v[0].x), "+v"(v[0].y), "+v"(v[0].z), "+v"(v[0].w), "+v"(v[1].x), "+v"(v[1].y),
                       "+v"(v[1].z), "+v"(v[1].w), "+v"(v[2].x), "+v"(v[2].y), "+v"(v[2].z), "+v"(v[2].w),
                       "+v"(v[3].x), "+v"(v[3].y), "+v"(v[3].z), "+v"(v[3].w));
}

// hook(g) runs at the start of group g (for every g with 4g < D): the caller's way
// of spreading memory instructions over the compute instead of issuing them in a
// burst that fills the memory pipeline and blocks the waves at issue.
template <int DMAX, int BUF, typename Hook>
__device__ __forceinline__ void sched_steps(const LayerArgs& a, uint32_t lds_base, int lane, const SchedNeuron<DMAX>& n,
                                            float (&acc)[SCHED_T], Hook&& hook) {
    // Steps in groups of 4; the reads of group g+1 are issued before the FMAs of
    // group g (ping-pong register sets).  Steps past D are padding (weight 0, a
    // conflict-free read), so reading one group ahead is always safe.
    static_assert(DMAX % 4 == 0, "groups of 4");
    // D is re-read through an empty asm each time, so the compiler compares it per
    // group (two scalar instructions) instead of keeping a mask per group alive
    int D = n.D;
    __asm__ volatile("" : "+s"(D));
    float4 v[2][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[0][u] = lds_read16(n.off[u] + BUF * 1024);
#pragma unroll
    for (int g = 0; g < DMAX / 4; ++g) {
        if (4 * g < D) {
            hook(g);
            if (g + 1 < DMAX / 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) v[(g + 1) & 1][u] = lds_read16(n.off[4 * (g + 1) + u] + BUF * 1024);
                // one wait for the whole group (the 4 reads just issued stay in flight):
                // the empty asm consumes the group's values, so the compiler waits for
                // all four at once instead of before each step's FMAs
                consume16(v[g & 1]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int st = 4 * g + u;
                const float4 c = v[g & 1][u];
                acc[0] = fmaf(n.wv[st], c.x, acc[0]);
                acc[1] = fmaf(n.wv[st], c.y, acc[1]);
                acc[2] = fmaf(n.wv[st], c.z, acc[2]);
                acc[3] = fmaf(n.wv[st], c.w, acc[3]);
            }
        }
    }
    if (D > DMAX) {
        // the LDS and memory forms are separate loops so that the LDS one never waits
        // on outstanding memory operations (the staging of the next tile)
        if (n.ovf != ~0u) {
            // four steps at a time: their pairs, then their slots, then the FMAs (two
            // LDS latencies per four steps); a group's steps past D re-read the last
            // pair and add nothing
            for (int st0 = DMAX; st0 < D; st0 += 4) {
                uint2 e[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    e[u] = lds_read8(n.ovf + (uint32_t)(min(st0 + u, D - 1) - DMAX) * 512u + 8u * (uint32_t)lane);
                float4 c[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) c[u] = lds_read16(e[u].x + BUF * 1024);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float w = st0 + u < D ? __uint_as_float(e[u].y) : 0.f;
                    acc[0] = fmaf(w, c[u].x, acc[0]);
                    acc[1] = fmaf(w, c[u].y, acc[1]);
                    acc[2] = fmaf(w, c[u].z, acc[2]);
                    acc[3] = fmaf(w, c[u].w, acc[3]);
                }
            }
        } else {
            for (int st = DMAX; st < D; ++st) {
                const uint32_t e = a.ent[(size_t)st * (a.nblk * 64) + n.slot];
                const float w = n.weight_of(a, e, st);
                const float4 c = lds_read16(lds_base + ((e >> 5) & 0x03ffffffu) + BUF * 1024);
                acc[0] = fmaf(w, c.x, acc[0]);
                acc[1] = fmaf(w, c.y, acc[1]);
                acc[2] = fmaf(w, c.z, acc[2]);
                acc[3] = fmaf(w, c.w, acc[3]);
            }
        }
    }
}

// The scheduled layer over R rows (tiles of 4 rows; see the comment above).
// Per tile: wait for this wave's block copies of the tile and turn its blocks
// into [id][row]; (lockstep); meet at the barrier; advance the liveness pipeline
// and store the previous tile's outputs; compute, issuing the next tile's block
// copies into the other buffer one per compute group; stage the outputs.
// No memory load is waited for inside the compute: the row ids of a tile are
// fetched two tiles ahead, output stores are issued a tile late, and the row
// liveness (LINEAR = false, with a work list or alive flags) runs as a pipeline
// on wave 0: tile t's combined row bits are added to its tile word at tile t+1,
// the sum is read at tile t+2 (alive flags, zeroing of dead rows, list slot
// reservation), the list entries are written at tile t+3, and whatever is left
// drains after the last tile.
template <int NT, int DMAX, bool LINEAR = false, int DMAX1 = DMAX>
__device__ __forceinline__ void run_layer_sched(const LayerArgs& a, float* __restrict__ lds, int R) {
    constexpr int T = SCHED_T;
    constexpr int WAVES = NT / 64;
    const int N = a.N;
    const SchedLds L(lds, N);
    unsigned* s_bits = L.scalars;                         // [3] row bits of the last three tiles
    int* s_pin = reinterpret_cast<int*>(L.scalars) + 8;   // [2][4] input rows of coming tiles
    int* s_pout = reinterpret_cast<int*>(L.scalars) + 16; // [2][4] output rows (linear mode)
    int* s_prog = reinterpret_cast<int*>(L.scalars) + 24; // [4] the parts' progress words, a tile old
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int G = a.parts;
    const int b = blockIdx.x;
    const int x = b & 7, kk = b >> 3;
    const int p = kk % G;
    const int q = (kk / G) * 8 + x;
    const int S = (int)gridDim.x / G;
    const int ntiles = (R + T - 1) / T;
    if (q >= ntiles) return;                         // uniform over the workgroup
    // a part is 16 blocks of 64 neurons; wave w owns blocks 2w and 2w + 1 of it
    // (DMAX register steps for the even block, DMAX1 for the odd one)
    SchedNeuron<DMAX> n0;
    SchedNeuron<DMAX1> n1;
    n0.load(a, p * 16, p * 16 + 2 * wave, lane, L.base, L.ovf, lds, DMAX, DMAX1);
    n1.load(a, p * 16, p * 16 + 2 * wave + 1, lane, L.base, L.ovf, lds, DMAX, DMAX1);
    const bool live = !LINEAR && (a.list_out || a.alive);
    int* prog_q = (G > 1 && a.prog) ? a.prog + 4 * q : nullptr;   // this stream's progress words
    const unsigned tag = ((unsigned)a.layer & 0xfffu) << 20;
    // Row ids: lane l carries the id of tile row l % 4.  With a work list (and in linear
    // mode with an output row map) the ids of the tile after next are copied by wave 0
    // into an LDS ring with asynchronous copies, so no register waits on a memory load
    // inside the loop.
    auto pos_of = [&](int tile) -> int {
        const int pos = tile * T + (lane & 3);
        return pos < R ? pos : tile * T;             // padding rows repeat the tile's first row
    };
    auto prefetch = [&](int tile, int slot) {
        if (wave == 0 && lane < T) {
            const int pp = pos_of(tile);
            if (a.list_in) lds_copy4(a.list_in + pp, s_pin + 4 * slot);
            if (LINEAR && a.rows_out) lds_copy4(a.rows_out + pp, s_pout + 4 * slot);
        }
    };
    // rows of a tile whose ids are in ring slot `slot` (valid after the barrier that follows the copy)
    auto in_row = [&](int tile, int slot) -> int { return a.list_in ? s_pin[4 * slot + (lane & 3)] : a.row_base + pos_of(tile); };
    // the input row of tile row t (the block copies' lanes take row lane / 16)
    auto in_row_t = [&](int tile, int slot, int t) -> int {
        const int pos = tile * T + t;
        return a.list_in ? s_pin[4 * slot + t] : a.row_base + (pos < R ? pos : tile * T);
    };
    auto out_row = [&](int tile, int slot) -> int {
        return (LINEAR && a.rows_out) ? s_pout[4 * slot + (lane & 3)] : in_row(tile, slot);
    };
    // wave 0's liveness pipeline (see above): A = tile whose word add is in flight,
    // B = tile whose list slots are being reserved.  The returned values are read
    // first, unconditionally, while nothing else is outstanding; only then are new
    // stores and atomics issued.
    int tA = -1, rowA = 0, tB = -1, rowB = 0;
    unsigned mineA = 0u, oldA = 0u, maskB = 0u;
    int baseB = 0;
    auto advance = [&](int tile_new, int row_new, unsigned mine_new) {
        const unsigned old = __builtin_amdgcn_readfirstlane(oldA);
        const int base = __builtin_amdgcn_readfirstlane(baseB);
        // B: write the list entries of the tile whose slots were reserved
        if (tB >= 0) {
            if (lane < T && ((maskB >> lane) & 1u)) a.list_out[base + __popc(maskB & ((1u << lane) - 1u))] = rowB;
            tB = -1;
        }
        // A: the word sum is back; the part that completed the tile publishes it
        if (tA >= 0) {
            if ((old >> 16) == (unsigned)(G - 1)) {
                const unsigned full = (old | (mineA << (4 * p))) & 0xffffu;
                const int nv = min(T, R - tA * T);
                const unsigned all = (full | (full >> 4) | (full >> 8) | (full >> 12)) & ((1u << nv) - 1u);
                if (G > 1 && lane == 0) atomicExch(&a.tile_bits[tA], 0);
                if (a.alive && lane < nv) a.alive[rowA] = ((all >> lane) & 1u) ? 1 : a.dead_mark;
                if (a.list_out && all) {
                    baseB = lane == 0 ? atomicAdd(a.cnt_out, __popc(all)) : 0;
                    maskB = all;
                    rowB = rowA;
                    tB = tA;
                }
            }
            tA = -1;
        }
        // the new tile: add this part's row bits to its word
        if (tile_new >= 0) {
            mineA = mine_new;
            oldA = 0u;
            if (G > 1 && lane == 0)
                oldA = (unsigned)atomicAdd(&a.tile_bits[tile_new], (int)((1u << 16) | (mine_new << (4 * p))));
            tA = tile_new;
            rowA = row_new;
        }
    };

    if (tid == 0) { s_bits[0] = 0u; s_bits[1] = 0u; s_bits[2] = 0u; }
    // the ids of tiles q and q + S come through the ring too, so no register in the
    // loop ever waits on a row-id load
    prefetch(q, 0);
    if (q + S < ntiles) prefetch(q + S, 1);
    __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
    __syncthreads();
    int row_c = in_row(q, 0), orow_c = out_row(q, 0);   // rows of the tile being computed next
    int rowx_c = in_row_t(q, 0, lane >> 4);
    {
        auto c0 = L.cursor<WAVES>(a.yin, rowx_c, lane, wave, 0, true);
        c0.finish();
    }
    int tile_p = -1, row_p = 0, orow_p = 0;          // the previous tile (outputs not yet stored)
    // Each wave stages its own outputs (its two blocks: neurons wbase .. wbase+127,
    // 4 rows) in a private 2 KB of LDS and stores them with 16-byte stores after the
    // next barrier; no other wave touches that area.  A row that dies is not cleared
    // here: the other parts of its tile may still be reading it, and no kernel writes
    // its own input (its alive flag says whether the finalize pass must clear it).
    const int wbase = p * SCHED_PART + 128 * wave;
    float* wout = L.out + 512 * wave;
    auto store_own = [&]() {
        const int nv = min(T, R - tile_p * T);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int e = (k * 64 + lane) * 4;
            const int t = e >> 7;                    // rows 2k (lanes 0..31) and 2k + 1
            const int col = e & 127;
            // rows 2k and 2k + 1 are held by lanes 2k and 2k + 1 (lane t: tile row t)
            const int rsrc = LINEAR ? orow_p : row_p;
            const int ra = __builtin_amdgcn_readlane(rsrc, 2 * k), rb = __builtin_amdgcn_readlane(rsrc, 2 * k + 1);
            const int ro = (lane >> 5) ? rb : ra;
            if (t < nv && wbase + col < N) {
                const size_t o = (size_t)ro * N + wbase + col;
                const float4 v = *reinterpret_cast<const float4*>(wout + e);
                *reinterpret_cast<float4*>(a.yout + o) = v;
                if (a.ycopy) *reinterpret_cast<float4*>(a.ycopy + o) = v;
            }
        }
    };
    int it = 0;
    for (int tile = q; tile < ntiles; tile += S, ++it) {
        const int buf = it & 1;
        const int slot = it % 3;                     // row-bit word of this tile
        __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
        L.transpose<WAVES, 8>(wave, lane, buf);      // this wave's blocks of the tile, now landed
        if (prog_q && tid == 0) {
            __hip_atomic_store(prog_q + p, (int)(tag | (unsigned)it), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (it > SCHED_AHEAD) {
                int mn = it;
                for (int pp = 0; pp < G; ++pp) mn = min(mn, part_progress(s_prog[pp], tag));
                if (mn < it - SCHED_AHEAD) {
                    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                    while (__builtin_amdgcn_s_memrealtime() - t0 < SCHED_WAIT_TICKS) {
                        __builtin_amdgcn_s_sleep(1);
                        mn = it;
                        for (int pp = 0; pp < G; ++pp)
                            mn = min(mn, part_progress(__hip_atomic_load(prog_q + pp, __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_AGENT), tag));
                        if (mn >= it - SCHED_AHEAD) break;
                    }
                }
            }
        }
        // The tile has landed in buffer buf; every wave is done with the other buffer
        // (the previous tile), which the next tile's copies now fill.
        __syncthreads();
        // (register moves of loop-carried row ids first, while nothing is outstanding)
        const int row_now = row_c, orow_now = orow_c;
        if (tile_p >= 0) {
            const unsigned mine = live ? s_bits[(it + 2) % 3] : 0xfu;
            if (live && wave == 0) advance(tile_p, row_p, mine);   // before any store: nothing outstanding
            store_own();
        }
        // the word of two tiles ago: read by every wave before this barrier, next
        // written after the next one
        if (tid == 0) s_bits[(it + 1) % 3] = 0u;
        const bool more = tile + S < ntiles;
        if (more) {
            // ring slot (it + 1) & 1 holds tile + S's ids (copied a tile ago, waited above)
            row_c = in_row(tile + S, buf ^ 1);
            rowx_c = in_row_t(tile + S, buf ^ 1, lane >> 4);
            orow_c = out_row(tile + S, buf ^ 1);
        }
        if (tile + 2 * S < ntiles) prefetch(tile + 2 * S, buf);
        if (prog_q && wave == 0 && lane < G) lds_copy4_coherent(prog_q + lane, s_prog + lane);
        // the next tile's block copies, one per compute group
        auto cur = L.cursor<WAVES>(a.yin, rowx_c, lane, wave, buf ^ 1, more);
        auto issue = [&](int) { cur.issue(); };
        float acc0[T] = {0.f, 0.f, 0.f, 0.f}, acc1[T] = {0.f, 0.f, 0.f, 0.f};
        if (buf == 0) {
            sched_steps<DMAX, 0>(a, L.base, lane, n0, acc0, issue);
            sched_steps<DMAX1, 0>(a, L.base, lane, n1, acc1, issue);
        } else {
            sched_steps<DMAX, 1>(a, L.base, lane, n0, acc0, issue);
            sched_steps<DMAX1, 1>(a, L.base, lane, n1, acc1, issue);
        }
        cur.finish();
        unsigned bits = 0u;
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const float o0 = LINEAR ? acc0[t] : fminf(fmaxf(acc0[t] + n0.bj, 0.f), a.clamp);
            const float o1 = LINEAR ? acc1[t] : fminf(fmaxf(acc1[t] + n1.bj, 0.f), a.clamp);
            if (n0.j >= 0) wout[t * 128 + (n0.j - wbase)] = o0;
            if (n1.j >= 0) wout[t * 128 + (n1.j - wbase)] = o1;
            bits |= ((o0 != 0.f && n0.j >= 0) || (o1 != 0.f && n1.j >= 0)) ? (1u << t) : 0u;
        }
        if (live) {
            // row bits of this part: its waves meet in LDS (read after the next barrier)
            unsigned wbits = 0u;                     // the wave's row bits, from one ballot per row
#pragma unroll
            for (int t = 0; t < T; ++t) wbits |= __ballot((bits >> t) & 1u) ? (1u << t) : 0u;
            if (lane == 0 && wbits) atomicOr(&s_bits[slot], wbits);
        }
        tile_p = tile;
        row_p = row_now;
        orow_p = orow_now;
    }
    // drain: the last tile's outputs and the rest of the liveness pipeline
    __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
    __syncthreads();
    const unsigned mine_last = live ? s_bits[(it - 1) % 3] : 0xfu;
    if (live && wave == 0) {
        advance(tile_p, row_p, mine_last);
        __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
        advance(-1, 0, 0u);
        __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
        advance(-1, 0, 0u);
    }
    store_own();
    __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
}

template <int NT, int DMAX>
__global__ __launch_bounds__(NT) void k_layer_sched(LayerArgs a) {
    extern __shared__ __align__(16) float lds[];
    const int R = a.cnt_in ? *a.cnt_in : a.nrows;
    run_layer_sched<NT, DMAX>(a, lds, R);
}

template <int NT, int DMAX>
__global__ __launch_bounds__(NT) void k_chain_sched(ChainArgs) {
    extern __shared__ __align__(16) float lds[];
    unsigned gen = 0u;
    for (int l = 0;; ++l) {
        {
            const ChainArgs c = reload_chain_args();
            if (l >= c.L) break;
            const int R = (l == 0 || !c.compaction) ? c.rows : ld_count(&c.cnt[l]);
            if (R == 0) break;
            const size_t npad = (size_t)c.nblk * 64;
            LayerArgs a = chain_layer_args(c, l, R);
            a.ent = c.ent + (size_t)l * npad * SCHED_DSTORE;
            a.lane_neuron = c.lane_neuron + (size_t)l * npad;
            a.wave_steps = c.wave_steps + (size_t)l * c.nblk;
            a.tile_bits = c.tile_bits;
            a.prog = c.prog;
            a.parts = c.parts;
            a.nblk = c.nblk;
            run_layer_sched<NT, DMAX>(a, lds, R);
        }
        const ChainArgs c = reload_chain_args();
        if (!grid_barrier(c.bar, gen, c.err, reinterpret_cast<int*>(lds + sched_tile_bytes(c.N) / 4) + 4)) return;
    }
}

// Input gradient through the transposed pattern: the scheduled kernel in linear
// mode (lane = input neuron, steps = its incoming edges, tile = the masked
// gradient G of 4 rows, no bias / clamp / liveness).
template <int NT, int DMAX0, int DMAX1>
__global__ __launch_bounds__(NT) void k_bwd_dy_sched(LayerArgs a) {
    extern __shared__ __align__(16) float lds[];
    const int R = a.cnt_in ? *a.cnt_in : a.nrows;
    run_layer_sched<NT, DMAX0, true, DMAX1>(a, lds, R);
}

// Weight and bias gradients with the forward schedule.  A workgroup of 1024
// lanes (16 waves, four per SIMD) owns a part of 1024 neurons; each lane owns one
// neuron and, for every step (one slot of its neuron), keeps
//   acc[st] = sum over its rows of G[r][j] * Y_l[r][id(st)]
// (rows in ascending order within its tile stream), so a stream's partial sums
// are deterministic.  The masked gradient G[r][j] = dY[r][j] [0 < Y_{l+1} < c]
// is also written out for the input-gradient pass.  Tiles of Y_l are staged like
// the forward kernel's (the next tile's copies spread over the compute groups);
// the Y_{l+1} and dY values a lane needs for a tile are loaded one tile ahead.
// Steps past DMAX keep their (offset, sum) pairs in the LDS overflow area (else
// in memory).  With one neuron per lane the sums fit in 128 registers, so four
// waves per SIMD hide the LDS latency.
template <int NT, int DMAX>
__global__ __launch_bounds__(NT) void k_bwd_dw_sched(SchedDwArgs a) {
    extern __shared__ __align__(16) float lds[];
    constexpr int T = SCHED_T;
    constexpr int WAVES = NT / 64;
    static_assert(WAVES == 16, "one block of 64 neurons per wave, 16 blocks per part");
    const int N = a.N;
    const SchedLds L(lds, N);
    const int R = *a.nrows;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int G = a.parts;
    const int b = blockIdx.x;
    const int x = b & 7, kk = b >> 3;
    const int p = kk % G;
    const int q = (kk / G) * 8 + x;
    const int S = (int)gridDim.x / G;
    const int ntiles = (R + T - 1) / T;
    // a stream with no tile writes no partials (the reduction stops before it)
    if (q >= ntiles) return;                         // uniform over the workgroup
    const int blk = p * 16 + wave;
    const bool have = blk < a.nblk;
    const int slot = blk * 64 + lane;
    const int j = have ? a.lane_neuron[slot] : -1;
    const int D = have ? __builtin_amdgcn_readfirstlane(a.wave_steps[blk]) : 0;
    uint32_t off[DMAX];
    float acc[DMAX];
    float accb = 0.f;
    {
        uint32_t e[DMAX];
#pragma unroll
        for (int st = 0; st < DMAX; ++st)
            e[st] = (have && st < D) ? a.ent[(size_t)st * (a.nblk * 64) + slot] : (0x80000000u | 31u);
#pragma unroll
        for (int st = 0; st < DMAX; ++st) {
            off[st] = L.base + ((e[st] >> 5) & 0x03ffffffu);
            acc[st] = 0.f;
        }
    }
#pragma unroll
    for (int st = 0; st < DMAX; ++st) __asm__ volatile("" : "+v"(off[st]));
    uint32_t ovf = ~0u;            // LDS address of the block's overflow (offset, sum) pairs, or ~0u
    if (D > DMAX) {
        // the part's blocks take the overflow area in block order
        int pre = 0;
        for (int b2 = p * 16; b2 < blk; ++b2) pre += max(0, __builtin_amdgcn_readfirstlane(a.wave_steps[b2]) - DMAX);
        if (pre + (D - DMAX) <= SCHED_OVF) {
            ovf = L.ovf + (uint32_t)pre * 512u;
            uint2* dst = reinterpret_cast<uint2*>(reinterpret_cast<char*>(lds) + (ovf - L.base)) + lane;
            for (int st = DMAX; st < D; ++st) {
                const uint32_t e2 = a.ent[(size_t)st * (a.nblk * 64) + slot];
                dst[(st - DMAX) * 64] = make_uint2(L.base + ((e2 >> 5) & 0x03ffffffu), __float_as_uint(0.f));
            }
        } else if (j >= 0) {
            // no room: those slots accumulate in memory, from zero
            float* pw = a.pdw + ((size_t)q * N + j) * K;
            for (int st = DMAX; st < D; ++st) {
                const uint32_t e2 = a.ent[(size_t)st * (a.nblk * 64) + slot];
                if (!(e2 & 0x80000000u)) pw[e2 & 31u] = 0.f;
            }
        }
    }
    float yo[T], dv[T];            // Y_{l+1} and dY of the lane's neuron for the next tile
    auto fetch = [&](int tile) {
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int r = tile * T + t;
            yo[t] = 0.f;
            dv[t] = 0.f;
            if (r < R && j >= 0) {
                const size_t o = (size_t)r * N + j;
                yo[t] = a.y_out[o];
                dv[t] = a.dy[o];
            }
        }
    };
    // rows of a tile are consecutive (padding positions repeat the tile's first row)
    auto row_of_t = [&](int tile, int t) -> int {
        const int pos = tile * T + t;
        return pos < R ? pos : tile * T;
    };
    if (q < ntiles) {
        auto c0 = L.cursor<WAVES>(a.y_in, row_of_t(q, lane >> 4), lane, wave, 0, true);
        c0.finish();
        fetch(q);
    }
    int it = 0;
    for (int tile = q; tile < ntiles; tile += S, ++it) {
        const int buf = it & 1;
        __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
        L.transpose<WAVES, 1>(wave, lane, buf);       // this wave's blocks of the tile, now landed
        __syncthreads();                             // tile in buffer buf; the other buffer is free
        // G of this tile from the values fetched a tile ago (before any copy is issued,
        // so reading them waits for nothing new)
        float g[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            g[t] = (yo[t] > 0.f && yo[t] < a.clamp) ? dv[t] : 0.f;
            accb += g[t];
            if (tile * T + t < R && j >= 0) a.g_out[(size_t)(tile * T + t) * N + j] = g[t];
        }
        const bool more = tile + S < ntiles;
        if (more) fetch(tile + S);
        // the next tile's block copies, one per compute group
        auto cur = L.cursor<WAVES>(a.y_in, row_of_t(tile + S, lane >> 4), lane, wave, buf ^ 1, more);
#pragma unroll
        for (int g4 = 0; g4 < DMAX / 4; ++g4) {
            if (4 * g4 < D) {
                cur.issue();
                float4 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = buf == 0 ? lds_read16(off[4 * g4 + u]) : lds_read16(off[4 * g4 + u] + 1024);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    float s = acc[4 * g4 + u];
                    s = fmaf(g[0], v[u].x, s);
                    s = fmaf(g[1], v[u].y, s);
                    s = fmaf(g[2], v[u].z, s);
                    s = fmaf(g[3], v[u].w, s);
                    acc[4 * g4 + u] = s;
                }
            }
        }
        cur.finish();
        if (D > DMAX) {
            if (ovf != ~0u) {
                for (int st = DMAX; st < D; ++st) {
                    const uint32_t pa = ovf + (uint32_t)(st - DMAX) * 512u + 8u * (uint32_t)lane;
                    const uint2 e2 = lds_read8(pa);
                    const float4 c = lds_read16(e2.x + 1024u * (uint32_t)buf);
                    float s = __uint_as_float(e2.y);
                    s = fmaf(g[0], c.x, s);
                    s = fmaf(g[1], c.y, s);
                    s = fmaf(g[2], c.z, s);
                    s = fmaf(g[3], c.w, s);
                    reinterpret_cast<float*>(reinterpret_cast<char*>(lds) + (pa - L.base))[1] = s;
                }
            } else if (j >= 0) {
                float* pw = a.pdw + ((size_t)q * N + j) * K;
                for (int st = DMAX; st < D; ++st) {
                    const uint32_t e2 = a.ent[(size_t)st * (a.nblk * 64) + slot];
                    if (e2 & 0x80000000u) continue;
                    const float4 c = lds_read16(L.base + ((e2 >> 5) & 0x03ffffffu) + 1024u * (uint32_t)buf);
                    float s = pw[e2 & 31u];
                    s = fmaf(g[0], c.x, s);
                    s = fmaf(g[1], c.y, s);
                    s = fmaf(g[2], c.z, s);
                    s = fmaf(g[3], c.w, s);
                    pw[e2 & 31u] = s;
                }
            }
        }
    }
    __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
    // Partials out.  A wave's 64 neurons are one contiguous block of 64 rows of 32 floats
    // in this stream's partials: staged in the wave's 1 KB of the output staging area in
    // 8 rounds of 8 neurons, they go out as contiguous 16-byte stores instead of scattered
    // 4-byte ones.  A block whose overflow sums live in memory writes its sums directly.
    // The entry pointer walks one step at a time behind an empty asm, so that the
    // compiler keeps one address instead of one 64-bit address per step.
    const bool direct = D > DMAX && ovf == ~0u;
    const int bbase = blk * 64;                    // first neuron of the block
    const int jl = j - bbase;                      // the block holds neurons bbase..bbase+63
    float* stg = L.out + 256 * wave;               // [8][32]
    const size_t es = (size_t)a.nblk * 64;         // step stride of the schedule entries
#pragma unroll 1
    for (int r = 0; r < 8; ++r) {
        __syncthreads();
        if (!direct && j >= 0 && (jl >> 3) == r) {
            const uint32_t* ep = a.ent + slot;
#pragma unroll
            for (int st = 0; st < DMAX; ++st) {
                if (st < D) {
                    const uint32_t e2 = *ep;
                    if (!(e2 & 0x80000000u)) stg[(jl & 7) * 32 + (e2 & 31u)] = acc[st];
                }
                ep += es;
                __asm__ volatile("" : "+v"(ep));
            }
            if (ovf != ~0u) {
                for (int st = DMAX; st < D; ++st) {
                    const uint32_t e2 = *ep;
                    const uint32_t pa = ovf + (uint32_t)(st - DMAX) * 512u + 8u * (uint32_t)lane;
                    if (!(e2 & 0x80000000u)) stg[(jl & 7) * 32 + (e2 & 31u)] = __uint_as_float(lds_read8(pa).y);
                    ep += es;
                }
            }
        }
        __syncthreads();
        // 8 neurons x 32 floats, one float4 per lane
        const int nr = bbase + 8 * r + (lane >> 3);
        if (!direct && have && nr < N)
            *reinterpret_cast<float4*>(a.pdw + ((size_t)q * N + nr) * K + 4 * (lane & 7)) =
                *reinterpret_cast<const float4*>(stg + 4 * lane);
    }
    if (j >= 0) {
        if (direct) {
            float* pw = a.pdw + ((size_t)q * N + j) * K;
            const uint32_t* ep = a.ent + slot;
#pragma unroll
            for (int st = 0; st < DMAX; ++st) {
                if (st < D) {
                    const uint32_t e2 = *ep;
                    if (!(e2 & 0x80000000u)) pw[e2 & 31u] = acc[st];
                }
                ep += es;
                __asm__ volatile("" : "+v"(ep));
            }
        }
        a.pdb[(size_t)q * N + j] = accb;
    }
}

// ---------------------------------------------------------------- small kernels
__global__ void k_chain_init(int32_t* cnt, int32_t L, int32_t rows, int32_t compaction, unsigned* bar, int32_t nbar) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= L; i += gridDim.x * blockDim.x)
        cnt[i] = (i == 0 || !compaction) ? rows : 0;
    if (bar)
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nbar; i += gridDim.x * blockDim.x) bar[i] = 0u;
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Parameter validation: bit 1 = id out of range, 2 = ids not strictly ascending,
// 4 = non-finite weight, 8 = non-finite bias.
__global__ void k_check_params(const int32_t* idx, const float* w, const float* b, int32_t N, int32_t L, int32_t* bad,
                               float* /*unused*/) {
    const int64_t neurons = (int64_t)N * L;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < neurons; n += (int64_t)gridDim.x * blockDim.x) {
        int flags = 0;
        int prev = -1;
        for (int k = 0; k < K; ++k) {
            const int v = idx[n * K + k];
            if (v < 0 || v >= N) flags |= 1;
            if (v <= prev) flags |= 2;
            prev = v;
            if (!isfinite(w[n * K + k])) flags |= 4;
        }
        if (!isfinite(b[n])) flags |= 8;
        if (flags) atomicOr(bad, flags);
    }
}

// flag_pos[0] |= 1 if any bias is > 0 or NaN (compaction would not be exact).
__global__ void k_max_bias(const float* b, int64_t n, int32_t* flag_pos) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = b[i];
        if (!(v <= 0.f)) atomicOr(flag_pos, 1);
    }
}

// MSE: dy = scale * (y - t); per-block partial sums of (y - t)^2 in a fixed order.
constexpr int MSE_NT = 256;
__global__ __launch_bounds__(MSE_NT) void k_mse(const float* y, const float* t, int64_t n, float* dy, float* partial,
                                                float scale) {
    __shared__ float s[MSE_NT];
    float acc = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * MSE_NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * MSE_NT) {
        const float d = y[i] - t[i];
        if (dy) dy[i] = scale * d;
        acc = fmaf(d, d, acc);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = MSE_NT / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0 && partial) partial[blockIdx.x] = s[0];
}

__global__ void k_mse_final(const float* partial, int32_t nparts, float* loss, float inv_n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nparts; ++i) s += partial[i];
        *loss = (float)(s * inv_n);
    }
}

// ---------------------------------------------------------------- variant table
#define SDNN_V(T, NT) {T, NT, 1, (const void*)&k_layer<T, NT, true>, (const void*)&k_chain<T, NT, true>, nullptr}
#define SDNN_VD(T, NT) {T, NT, 0, (const void*)&k_layer<T, NT, false>, (const void*)&k_chain<T, NT, false>, nullptr}
#define SDNN_VW(T, NT) {T, NT, 3, (const void*)&k_layer_wide<T, NT>, (const void*)&k_chain_wide<T, NT>, \
                        (const void*)&k_wide_pack<T>}
static const FwdVariant g_variants[] = {
    SDNN_V(1, 256),  SDNN_V(1, 512),  SDNN_V(1, 1024),
    SDNN_V(2, 256),  SDNN_V(2, 512),  SDNN_V(2, 1024),
    SDNN_V(4, 256),  SDNN_V(4, 512),  SDNN_V(4, 1024),
    SDNN_V(8, 256),  SDNN_V(8, 512),  SDNN_V(8, 1024),
    SDNN_V(16, 256), SDNN_V(16, 512), SDNN_V(16, 1024),
    SDNN_V(32, 256), SDNN_V(32, 512),
    SDNN_VD(1, 256), SDNN_VD(1, 512), SDNN_VD(1, 1024),
    SDNN_VD(2, 256), SDNN_VD(4, 256),
    {SCHED_T, SCHED_NT, 2, (const void*)&k_layer_sched<SCHED_NT, SCHED_DMAX>,
     (const void*)&k_chain_sched<SCHED_NT, SCHED_DMAX>, nullptr},
    SDNN_VW(8, 256),  SDNN_VW(8, 512),
    SDNN_VW(16, 256), SDNN_VW(16, 512),
    SDNN_VW(32, 256), SDNN_VW(32, 512),
    SDNN_VW(16, 1024), SDNN_VW(32, 1024),
    {1, ROW_NT, 4, (const void*)&k_layer_row, (const void*)&k_chain_row, nullptr},
    {1, ROW_NT, 5, (const void*)&k_layer_row_sched, (const void*)&k_chain_row_sched, nullptr},
    {2, ROW_NT, 6, (const void*)&k_layer_rowc<2>, (const void*)&k_chain_rowc<2>, nullptr},
    {4, ROW_NT, 6, (const void*)&k_layer_rowc<4>, (const void*)&k_chain_rowc<4>, nullptr},
    {2, ROW_NT, 7, (const void*)&k_layer_rowu<2>, (const void*)&k_chain_rowu<2>, nullptr},
    {4, ROW_NT, 7, (const void*)&k_layer_rowu<4>, (const void*)&k_chain_rowu<4>, nullptr},
};
#undef SDNN_V
#undef SDNN_VD
#undef SDNN_VW

int fwd_variant_count() { return (int)(sizeof(g_variants) / sizeof(g_variants[0])); }
const void* bwd_dw_sched_fn() { return (const void*)&k_bwd_dw_sched<2 * SCHED_NT, SCHED_DMAX>; }
const void* bwd_dy_sched_fn() { return (const void*)&k_bwd_dy_sched<SCHED_NT, SCHED_DMAX_T0, SCHED_DMAX_T1>; }
const FwdVariant& fwd_variant(int i) { return g_variants[i]; }

}  // namespace sdnn
