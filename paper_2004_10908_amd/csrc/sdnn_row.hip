// One-row-tile forward kernel for wide layers (2048 < N <= 16384 neurons).
//
// The layer rule is the one of the other forward kernels (paper, section "Large
// Sparse Neural Network Inference": y_{l+1}[r][j] = min(c, max(0, sum_k w[j][k]
// y_l[r][idx[j][k]] + b[j]))), summed with fused multiply-adds, then the bias.  In
// ascending slot order (plan variant 4) its outputs are bitwise equal to the
// streamed-weight and wide-layer kernels; in the bank-scheduled order (variant 5)
// each neuron's order is fixed at create time, so results are deterministic.
//
// Why this shape.  At N = 16384 a row of activations is 64 KB: two rows fit LDS
// (160 KB) as a double buffer, four do not.  The other wide kernels read each
// neuron's 32 (id, weight) pairs again for every row tile, and gather the inputs
// from the cache hierarchy; here the weights stay in registers for the whole
// layer and every gather is an LDS read:
//  * a workgroup of 1024 lanes owns a "part" of ROW_PART = 2048 consecutive
//    neurons, two per lane; each lane keeps its neurons' 32 weights and 32 input
//    offsets (16-bit LDS byte offsets, two per register) in registers, loaded once
//    per layer, in ascending slot order or (plan variant 5) in the create-time
//    order that keeps the 32 lanes of each half-wave on distinct LDS banks
//    (sdnn_rowsched.hip); the sum runs in that order;
//  * G = ceil(N / 2048) parts share each row ("tile" of one row).  Workgroup b
//    serves part (b / 8) % G of tile stream ((b / 8) / G) * 8 + b % 8, so the G
//    parts of a row run on one XCD (blockIdx % 8) and the row they all stage is
//    read from HBM once and served to the others by that XCD's L2;
//  * the next row arrives in the other buffer through asynchronous 16-byte
//    global->LDS copies (a wave copies 1 KB per instruction, in row order, so the
//    LDS buffer is the row itself: no transpose) issued between the compute steps;
//  * a slot read is one 4-byte LDS read whose address is built from the packed
//    offset and the buffer base by one byte permute.
// Outputs go through a per-part LDS stage and leave as 16-byte stores of the
// part's slice of the row.  Row liveness: the waves OR their outputs' nonzero
// bits in LDS, and the part adds (1 << 16) | bit to the row's word; the part that
// completes the count (G arrivals) writes the alive flag, takes a slot in the next
// work list and resets the word.  Those atomics run as a pipeline on wave 0 (issued
// one row, their returned values read the next), so no wave waits on them.
// Dead rows are never written here: the finalize pass clears them where needed
// (their alive flag says so), so no kernel writes its own input rows.
#include <type_traits>
#include <utility>

#include "sdnn_internal.hpp"
#include "sdnn_device.hpp"

namespace sdnn {

namespace {

constexpr uint32_t ROW_S_BITS = ROW_SCAL;          // [2] this part's row bit of the last two tiles
constexpr uint32_t ROW_S_RING = ROW_SCAL + 16;     // [3] row ids of coming tiles
constexpr uint32_t ROW_S_OK = ROW_SCAL + 64;       // grid-barrier flag of the persistent chain

// A lane's resident neuron: weights and packed LDS byte offsets of its 32 slots
// (slot 2i in the low half of o[i], slot 2i + 1 in the high half).
struct RowNeuron {
    float w[K];
    uint32_t o[K / 2];
    float bj;
    int j;      // neuron id, -1 past N
};

// With a slot order (PERM), step s reads slot row_perm[j][s] (the create-time
// bank schedule); without one, step s reads slot s (ascending ids).
template <bool PERM>
__device__ __forceinline__ void row_load(const LayerArgs& a, int j, RowNeuron& n) {
    n.j = j < a.N ? j : -1;
    if (PERM && n.j >= 0) {
        const uint4* pp = reinterpret_cast<const uint4*>(a.row_perm + (size_t)j * K);
        const uint4 p0 = pp[0], p1 = pp[1];
        const uint32_t pw[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
        const int32_t* ip = a.idx + (size_t)j * K;
        const float* wp = a.w + (size_t)j * K;
        uint32_t off[K];
#pragma unroll
        for (int s = 0; s < K; ++s) {
            const int slot = (int)((pw[s >> 2] >> (8 * (s & 3))) & 31u);
            n.w[s] = wp[slot];
            off[s] = (uint32_t)ip[slot] << 2;
        }
#pragma unroll
        for (int q = 0; q < K / 2; ++q) n.o[q] = off[2 * q] | (off[2 * q + 1] << 16);
        n.bj = a.b[j];
    } else if (n.j >= 0) {
        const int4* ip = reinterpret_cast<const int4*>(a.idx + (size_t)j * K);
        const float4* wp = reinterpret_cast<const float4*>(a.w + (size_t)j * K);
#pragma unroll
        for (int q = 0; q < K / 4; ++q) {
            const int4 iv = ip[q];
            const float4 wv = wp[q];
            n.w[4 * q + 0] = wv.x;
            n.w[4 * q + 1] = wv.y;
            n.w[4 * q + 2] = wv.z;
            n.w[4 * q + 3] = wv.w;
            n.o[2 * q + 0] = ((uint32_t)iv.x << 2) | ((uint32_t)iv.y << 18);
            n.o[2 * q + 1] = ((uint32_t)iv.z << 2) | ((uint32_t)iv.w << 18);
        }
        n.bj = a.b[j];
    } else {
#pragma unroll
        for (int s = 0; s < K; ++s) n.w[s] = 0.f;
#pragma unroll
        for (int s = 0; s < K / 2; ++s) n.o[s] = 0u;
        n.bj = 0.f;
    }
}

// LDS address of slot s in the buffer at byte `buf` (a multiple of 65536): the
// slot's 16-bit offset in the low half, the buffer's upper half kept.
template <int S>
__device__ __forceinline__ uint32_t row_addr(const RowNeuron& n, uint32_t buf) {
    return __builtin_amdgcn_perm(buf, n.o[S >> 1], (S & 1) ? 0x07060302u : 0x07060100u);
}

// Both neurons over all 32 slots of the row in buffer `buf`, RS slots at a time:
// the reads of group g + 1 are issued before the FMAs of group g, and an empty asm
// with a memory clobber after each group keeps the compiler from hoisting every
// read of the row to the top (which would hold 64 results in registers).
// hook(g) runs before group g (the next row's copies go there).
template <int RS, int G>
__device__ __forceinline__ void row_reads(const RowNeuron& n0, const RowNeuron& n1, uint32_t buf,
                                          float (&r)[2 * RS]) {
#pragma unroll
    for (int u = 0; u < RS; ++u) {
        r[2 * u] = row_lds_read(__builtin_amdgcn_perm(buf, n0.o[(RS * G + u) >> 1],
                                                      ((RS * G + u) & 1) ? 0x07060302u : 0x07060100u));
        r[2 * u + 1] = row_lds_read(__builtin_amdgcn_perm(buf, n1.o[(RS * G + u) >> 1],
                                                          ((RS * G + u) & 1) ? 0x07060302u : 0x07060100u));
    }
}

template <int RS, int G>
__device__ __forceinline__ void row_fmas(const RowNeuron& n0, const RowNeuron& n1, const float (&r)[2 * RS],
                                         float& acc0, float& acc1) {
#pragma unroll
    for (int u = 0; u < RS; ++u) {
        acc0 = fmaf(n0.w[RS * G + u], r[2 * u], acc0);
        acc1 = fmaf(n1.w[RS * G + u], r[2 * u + 1], acc1);
    }
    __asm__ volatile("" : "+v"(acc0), "+v"(acc1) : : "memory");
}

template <int RS, int G, typename Hook>
__device__ __forceinline__ void row_group(const RowNeuron& n0, const RowNeuron& n1, uint32_t buf, float& acc0,
                                          float& acc1, float (&v)[2][2 * RS], Hook& hook) {
    hook(G);
    if constexpr (G + 1 < K / RS) row_reads<RS, G + 1>(n0, n1, buf, v[(G + 1) & 1]);
    row_fmas<RS, G>(n0, n1, v[G & 1], acc0, acc1);
    if constexpr (G + 1 < K / RS) row_group<RS, G + 1>(n0, n1, buf, acc0, acc1, v, hook);
}

// RS: slots per group.  Four (eight reads in flight per wave) is faster than two
// (S3 merged graph 546 against 580 ms), in the per-layer launch and, since the chain
// reads its arguments again per layer, in the persistent chain.
template <int RS, typename Hook>
__device__ __forceinline__ void row_steps(const RowNeuron& n0, const RowNeuron& n1, uint32_t buf, float& acc0,
                                          float& acc1, Hook&& hook) {
    float v[2][2 * RS];
    row_reads<RS, 0>(n0, n1, buf, v[0]);
    row_group<RS, 0>(n0, n1, buf, acc0, acc1, v, hook);
}

}  // namespace

// One layer over the R rows of the work list (see the comment at the top).
template <bool PERM, int RS>
__device__ __forceinline__ void run_layer_row(const LayerArgs& a, int R) {
    const int N = a.N;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int WAVES = ROW_NT / 64;
    const int G = a.row_parts;
    if (G < 1) return;                                 // (never: the host sets ceil(N / ROW_PART))
    const int b = blockIdx.x, x = b & 7, kk = b >> 3;
    const int spx = (int)(gridDim.x >> 3) / G;        // tile streams per XCD group
    if (kk >= spx * G) return;                         // no part of any stream (uniform)
    const int p = kk % G;
    const int q = (kk / G) * 8 + x;
    const int S = spx * 8;
    if (q >= R) return;
    const int ntile = (R - q + S - 1) / S;             // this stream's tiles: positions q, q + S, ...
    const int pbase = p * ROW_PART;

    const lds_ptr<unsigned> s_bits = lds_at<unsigned>(ROW_S_BITS);
    const lds_ptr<int> s_ring = lds_at<int>(ROW_S_RING);
    const lds_ptr<float> stage = lds_at<float>(ROW_STAGE);   // [2][ROW_PART]

    RowNeuron n0, n1;
    row_load<PERM>(a, pbase + wave * 64 + lane, n0);
    row_load<PERM>(a, pbase + WAVES * 64 + wave * 64 + lane, n1);
#pragma unroll
    for (int s = 0; s < K; ++s) __asm__ volatile("" : "+v"(n0.w[s]), "+v"(n1.w[s]));   // keep resident
#pragma unroll
    for (int s = 0; s < K / 2; ++s) __asm__ volatile("" : "+v"(n0.o[s]), "+v"(n1.o[s]));

    const int ncopy = (N + 255) / 256;                 // 1 KB copies per row (the last may be partial)
    const int mycopies = wave < ncopy ? (ncopy - wave + WAVES - 1) / WAVES : 0;
    auto pos_row = [&](int i) -> int { return a.row_base + q + i * S; };   // identity work list
    // row ids of tile i come through the LDS ring when there is a work list
    auto prefetch = [&](int i) {
        if (a.list_in && wave == 0 && lane == 0) row_copy4(a.list_in + q + i * S, ROW_S_RING + 4u * (uint32_t)(i % 3));
    };
    auto ring_row = [&](int i) -> int {
        return a.list_in ? __builtin_amdgcn_readfirstlane(s_ring[i % 3]) : pos_row(i);
    };
    // copies of a row (global address src) into the buffer at byte `buf`: this wave's
    // k-th copy.  The row address and the wave index are opaque to the compiler, so
    // it recomputes each copy's address from them instead of holding one 64-bit
    // address per copy across the tile loop (in the persistent chain those were
    // spilled to VGPR lanes and read back one v_readlane at a time: 1.65 x the time
    // per layer)
    const uint64_t ybase = uniform_ptr(a.yin);
    auto row_src = [&](int row) -> uint64_t {
        uint64_t s = ybase + 4ull * (uint64_t)(uint32_t)row * (uint64_t)(uint32_t)N;
        __asm__ volatile("" : "+s"(s));
        return s;
    };
    auto copy = [&](uint64_t src, uint32_t buf, int k) {
        int w = wave;
        __asm__ volatile("" : "+s"(w));
        const int c = w + k * WAVES;
        if (c * 256 + 4 * lane < N) row_copy16(src + 1024ull * (uint32_t)c, 16u * (uint32_t)lane, buf + 1024u * (uint32_t)c);
    };

    // wave 0's liveness pipeline: A = tile whose word add is in flight, B = tile
    // whose work-list slot is being reserved
    int posA = -1, rowA = 0, posB = -1, rowB = 0;
    unsigned bitA = 0u, retA = 0u;
    int retB = 0;
    auto advance = [&](int pos_new, int row_new, unsigned bit_new) {
        const unsigned oldA = (unsigned)__builtin_amdgcn_readfirstlane((int)retA);
        const int base = __builtin_amdgcn_readfirstlane(retB);
        if (posB >= 0) {
            if (lane == 0) a.list_out[base] = rowB;
            posB = -1;
        }
        if (posA >= 0) {
            if ((int)(oldA >> 16) == G - 1) {          // this part completed the row
                const bool any = ((oldA & 0xffffu) + bitA) != 0u;
                if (lane == 0) {
                    if (G > 1) atomicExch(&a.row_words[posA], 0);
                    if (a.alive) a.alive[rowA] = any ? 1 : a.dead_mark;
                }
                if (any && a.list_out) {
                    retB = lane == 0 ? atomicAdd(a.cnt_out, 1) : 0;
                    rowB = rowA;
                    posB = posA;
                }
            }
            posA = -1;
        }
        if (pos_new >= 0) {
            retA = 0u;
            if (G > 1 && lane == 0) retA = (unsigned)atomicAdd(&a.row_words[pos_new], (int)((1u << 16) | bit_new));
            bitA = bit_new;
            rowA = row_new;
            posA = pos_new;
        }
    };
    // the previous tile's outputs, from its stage, as 16-byte stores of the part's slice
    auto store_stage = [&](int row, int sbuf) {
        const int e = 4 * tid;
        if (e < ROW_PART && pbase + e < N) {
            const lds_ptr<const float> sp = lds_at<const float>(ROW_STAGE + 4u * (uint32_t)(sbuf * ROW_PART + e));
            const float4 v = make_float4(sp[0], sp[1], sp[2], sp[3]);
            const size_t o = (size_t)row * N + pbase + e;
            *reinterpret_cast<float4*>(a.yout + o) = v;
            if (a.ycopy) *reinterpret_cast<float4*>(a.ycopy + o) = v;
        }
    };

    if (tid == 0) { s_bits[0] = 0u; s_bits[1] = 0u; }
    prefetch(0);
    if (ntile > 1) prefetch(1);
    __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
    __syncthreads();
    int row_c = ring_row(0);
    {
        const uint64_t src = row_src(row_c);
        for (int k = 0; k < mycopies; ++k) copy(src, 0u, k);
    }
    int row_p = 0;
    for (int i = 0; i < ntile; ++i) {
        uint32_t buf = (uint32_t)(i & 1) * ROW_BUF_BYTES;
        // (an opaque buffer base: the slot addresses of both buffers are not all kept live)
        __asm__ volatile("" : "+s"(buf));
        __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");   // this wave's copies of row i have landed
        __syncthreads();                                        // everyone's have; buffer buf ^ 1 is free
        if (i > 0) {
            if (wave == 0) {
                const unsigned bit = s_bits[(i - 1) & 1];
                advance(q + (i - 1) * S, row_p, bit);           // before any store: nothing outstanding
                if (lane == 0) s_bits[(i - 1) & 1] = 0u;
            }
            store_stage(row_p, (i - 1) & 1);
        }
        const bool more = i + 1 < ntile;
        const int row_n = more ? ring_row(i + 1) : 0;
        if (i + 2 < ntile) prefetch(i + 2);
        const uint64_t nsrc = row_src(row_n);
        float acc0 = 0.f, acc1 = 0.f;
        auto hook = [&](int g) {
            if (more && g < mycopies) copy(nsrc, buf ^ ROW_BUF_BYTES, g);
        };
        row_steps<RS>(n0, n1, buf, acc0, acc1, hook);
        if (more)
            for (int k = K / RS; k < mycopies; ++k) copy(nsrc, buf ^ ROW_BUF_BYTES, k);
        const float y0 = fminf(fmaxf(acc0 + n0.bj, 0.f), a.clamp);
        const float y1 = fminf(fmaxf(acc1 + n1.bj, 0.f), a.clamp);
        const lds_ptr<float> st = stage + (i & 1) * ROW_PART;
        if (n0.j >= 0) st[n0.j - pbase] = y0;
        if (n1.j >= 0) st[n1.j - pbase] = y1;
        const bool nz = (n0.j >= 0 && y0 != 0.f) || (n1.j >= 0 && y1 != 0.f);
        if (__ballot(nz) != 0ull && lane == 0)
            __hip_atomic_fetch_or(s_bits + (i & 1), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        row_p = row_c;
        row_c = row_n;
    }
    // drain: the last tile's outputs and the rest of the liveness pipeline
    __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
    __syncthreads();
    if (wave == 0) {
        advance(q + (ntile - 1) * S, row_p, s_bits[(ntile - 1) & 1]);
        __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
        advance(-1, 0, 0u);
        __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
        advance(-1, 0, 0u);
    }
    store_stage(row_p, (ntile - 1) & 1);
    __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
    __syncthreads();                                   // the LDS is reused by the next layer
}

template <bool PERM>
__device__ __forceinline__ void chain_row() {
    int* s_ok = (int*)lds_at<int>(ROW_S_OK);
    unsigned gen = 0u;
    for (int l = 0;; ++l) {
        int R;
        {
            const ChainArgs c = reload_chain_args();
            if (l >= c.L) break;
            R = (l == 0 || !c.compaction) ? c.rows : ld_count(&c.cnt[l]);
            if (R == 0) break;
            LayerArgs a = chain_layer_args(c, l, R);
            a.row_parts = c.row_parts;
            a.row_words = c.row_words;
            a.row_perm = c.row_perm ? c.row_perm + (size_t)l * c.N * K : nullptr;
            run_layer_row<PERM, 4>(a, R);
        }
        const ChainArgs c = reload_chain_args();
        if (!grid_barrier(c.bar, gen, c.err, s_ok)) return;
    }
}

__global__ __launch_bounds__(ROW_NT) void k_layer_row(LayerArgs a) {
    run_layer_row<false, 4>(a, a.cnt_in ? *a.cnt_in : a.nrows);
}
__global__ __launch_bounds__(ROW_NT) void k_chain_row(ChainArgs) { chain_row<false>(); }
__global__ __launch_bounds__(ROW_NT) void k_layer_row_sched(LayerArgs a) {
    run_layer_row<true, 4>(a, a.cnt_in ? *a.cnt_in : a.nrows);
}
__global__ __launch_bounds__(ROW_NT) void k_chain_row_sched(ChainArgs) { chain_row<true>(); }

}  // namespace sdnn
