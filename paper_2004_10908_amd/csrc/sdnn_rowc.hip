// Chunked one-row-tile forward kernel for rows wider than one LDS buffer
// (16384 < N <= 65536 neurons, N a multiple of 2048).
//
// The layer rule is the one of the other forward kernels (paper, section "Large
// Sparse Neural Network Inference": y_{l+1}[r][j] = min(c, max(0, sum_k w[j][k]
// y_l[r][idx[j][k]] + b[j]))), each neuron's slots summed in ascending order with
// fused multiply-adds, then the bias, so its outputs are bitwise equal to the
// streamed-weight, wide-layer and ascending one-row-tile kernels.
//
// Why this shape.  At 65536 neurons a row of activations is 256 KB and fits no
// LDS; the wide-layer kernel gathers 128-byte slots of 32-row tiles (8 MB, twice
// an XCD's L2) from the cache hierarchy.  Here, as in the one-row-tile kernel, a
// workgroup of 1024 lanes keeps a part of 2048 neurons' weights and offsets in
// registers for the whole layer and reads its inputs from LDS, and the row is
// staged in C = 2 or 4 chunks of CW = N / C ids (at most 64 KB) through the two
// 64 KB buffers, so every read of a chunk is an LDS read:
//  * the neurons of a part are paired (create time, on the host: a neuron whose
//    slots crowd some chunks goes with one whose slots crowd the others, so that
//    each pair has about 64 / C slots in every chunk); lane l of the part holds
//    pair l, neurons A and B;
//  * the lane's 64 register positions are 64 / C per chunk: A's slots of the chunk
//    in ascending order, then B's, then padding (weight 0); a pair's slots past a
//    chunk's positions ("overflow", about one per pair) go to a per-workgroup list
//    in LDS as (weight, offset | owner << 16), read after the chunk's positions;
//  * one running sum walks a chunk's positions: at the position where B's slots
//    begin (per lane) it is stored as A's sum and B's sum is taken up, so each
//    neuron still sums its slots in ascending order (chunk by chunk, a chunk's
//    positions before its overflow entries);
//  * the lanes' register images (positions, pair words, overflow lists) are built
//    once per net by k_rowc_build, so a layer starts with coalesced loads of them;
//  * C chunk steps per row: wait for this wave's copies, barrier, compute the
//    chunk from one buffer while the next chunk (of this row, or the first chunk of
//    the next row) arrives in the other by asynchronous 16-byte global->LDS copies
//    issued between the compute groups; C is even, so chunk c always sits in
//    buffer c % 2;
//  * outputs, row liveness and the work list are handled as in the one-row-tile
//    kernel (per-part LDS stage, 16-byte stores of the part's slice, the pipelined
//    per-row word on wave 0).
// Values that do not change over the row loop but depend on the chunk (buffer base,
// chunk source address, the lane's switch position, copy counts) are passed through
// empty asm statements at each step, so the compiler forms them there instead of
// hoisting one copy per (chunk, position) out of the loop, which spilled.
#include <type_traits>

#include "sdnn_internal.hpp"
#include "sdnn_device.hpp"

namespace sdnn {

namespace {

constexpr int RC_WAVES = ROW_NT / 64;
constexpr uint32_t RC_S_BITS = ROW_SCAL;         // [2] this part's row bit of the last two rows
constexpr uint32_t RC_S_RING = ROW_SCAL + 16;    // [3] row ids of coming rows
constexpr uint32_t RC_S_OK = ROW_SCAL + 64;      // grid-barrier flag of the persistent chain

__device__ __forceinline__ uint32_t byte_of(uint32_t v, int c) { return (v >> (8 * c)) & 0xffu; }

// A lane's pair of neurons: 64 register positions (weights, and 16-bit LDS byte
// offsets within the chunk buffer, two per register), with per-chunk counts.
struct RowcLane {
    float w[64];
    uint32_t o[32];
    uint32_t split;    // byte c: positions of neuron A in chunk c (B's follow)
    uint32_t ocnt;     // byte c: overflow entries of chunk c
    uint32_t obase;    // LDS byte address of the lane's first overflow entry
    uint32_t jab;      // neurons A (low 16 bits) and B (high) within the part
    float ba, bb;
};

// The lane's image of one layer: coalesced loads (register word r of lane l at
// img[r * ROW_NT + l]), and the part's overflow list copied into LDS.
__device__ __forceinline__ void rowc_load(const LayerArgs& a, int p, int tid, RowcLane& n) {
    const uint32_t* img = a.rowc_img + (size_t)p * ROWC_IMG * ROW_NT + tid;
#pragma unroll
    for (int r = 0; r < 64; ++r) n.w[r] = __uint_as_float(img[(size_t)r * ROW_NT]);
#pragma unroll
    for (int r = 0; r < 32; ++r) n.o[r] = img[(size_t)(64 + r) * ROW_NT];
    const uint4 m = reinterpret_cast<const uint4*>(a.rowc_meta)[(size_t)p * ROW_NT + tid];
    n.jab = m.x;
    n.split = m.y;
    n.ocnt = m.z;
    n.obase = ROWC_OVF + 8u * m.w;
    n.ba = a.b[p * ROW_PART + (int)(m.x & 0xffffu)];
    n.bb = a.b[p * ROW_PART + (int)(m.x >> 16)];
    // the part's overflow list: ROWC_OVF_CAP entries of 8 bytes, 16 bytes per lane
    const uint4* src = reinterpret_cast<const uint4*>(a.rowc_ovf + (size_t)p * ROWC_OVF_CAP * 2);
    if (tid < ROWC_OVF_CAP / 2) {
        const uint4 e = src[tid];
        typedef unsigned v4u __attribute__((ext_vector_type(4)));
        v4u v;
        v.x = e.x;
        v.y = e.y;
        v.z = e.z;
        v.w = e.w;
        *lds_at<v4u>(ROWC_OVF + 16u * (uint32_t)tid) = v;
    }
}

// LDS address of position P (a constant once the loops are unrolled) in the chunk
// buffer at byte `buf` (0 or 65536).
__device__ __forceinline__ uint32_t rowc_addr(const RowcLane& n, int P, uint32_t buf) {
    return __builtin_amdgcn_perm(buf, n.o[P >> 1], (P & 1) ? 0x07060302u : 0x07060100u);
}

template <int C, int CH, int RS, int G>
__device__ __forceinline__ void rowc_reads(const RowcLane& n, uint32_t buf, float (&r)[RS]) {
    constexpr int PC = 64 / C;
#pragma unroll
    for (int u = 0; u < RS; ++u) r[u] = row_lds_read(rowc_addr(n, PC * CH + RS * G + u, buf));
}

// The switch from A's sum to B's at the lane's switch position: a compare and two
// selects per position (the position is opaque per chunk step, so the compares are
// made there, not hoisted out of the row loop as 64 live lane masks).
template <int C, int CH, int RS, int G>
__device__ __forceinline__ void rowc_fmas(const RowcLane& n, uint32_t splitc, const float (&r)[RS], float& cur,
                                          float& acca, float& accb) {
    constexpr int PC = 64 / C;
#pragma unroll
    for (int u = 0; u < RS; ++u) {
        const int k = RS * G + u;
        const bool sw = (uint32_t)k == splitc;
        acca = sw ? cur : acca;
        cur = sw ? accb : cur;
        cur = fmaf(n.w[PC * CH + k], r[u], cur);
    }
    __asm__ volatile("" : "+v"(cur), "+v"(acca), "+v"(accb) : : "memory");
}

template <int C, int CH, int RS, int G, typename Hook>
__device__ __forceinline__ void rowc_group(const RowcLane& n, uint32_t buf, uint32_t splitc, float& cur, float& acca,
                                           float& accb, float (&v)[2][RS], Hook& hook) {
    constexpr int PC = 64 / C;
    hook(G);
    if constexpr (G + 1 < PC / RS) rowc_reads<C, CH, RS, G + 1>(n, buf, v[(G + 1) & 1]);
    rowc_fmas<C, CH, RS, G>(n, splitc, v[G & 1], cur, acca, accb);
    if constexpr (G + 1 < PC / RS) rowc_group<C, CH, RS, G + 1>(n, buf, splitc, cur, acca, accb, v, hook);
}

// Chunk CH of the row in the buffer at `buf`: its positions, then its overflow entries.
template <int C, int CH, int RS, typename Hook>
__device__ __forceinline__ void rowc_chunk(const RowcLane& n, uint32_t buf, float& acca, float& accb, Hook&& hook) {
    constexpr int PC = 64 / C;
    uint32_t splitc = byte_of(n.split, CH);          // PC: no switch in this chunk
    __asm__ volatile("" : "+v"(splitc));
    float cur = acca;
    float v[2][RS];
    rowc_reads<C, CH, RS, 0>(n, buf, v[0]);
    rowc_group<C, CH, RS, 0>(n, buf, splitc, cur, acca, accb, v, hook);
    // no switch to B in this chunk (A took every position): the running sum is A's
    const bool none = splitc == (uint32_t)PC;
    acca = none ? cur : acca;
    accb = none ? accb : cur;
    const int cnt = (int)byte_of(n.ocnt, CH);
    uint32_t ea = n.obase;
#pragma unroll
    for (int c = 0; c < CH; ++c) ea += 8u * byte_of(n.ocnt, c);
    for (int e = 0; e < cnt; ++e) {
        typedef unsigned v2u __attribute__((ext_vector_type(2)));
        const v2u en = *lds_at<v2u>(ea + 8u * (uint32_t)e);
        const float x = row_lds_read(buf | (en.y & 0xffffu));
        const float wv = __uint_as_float(en.x);
        if (en.y >> 16)
            accb = fmaf(wv, x, accb);
        else
            acca = fmaf(wv, x, acca);
    }
}

}  // namespace

// One layer over the R rows of the work list.
template <int C, int RS>
__device__ __forceinline__ void run_layer_rowc(const LayerArgs& a, int R) {
    const int N = a.N;
    const int CW = N / C;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int G = a.row_parts;
    if (G < 1) return;                                 // (never: the host sets N / ROW_PART)
    const int b = blockIdx.x, x = b & 7, kk = b >> 3;
    const int spx = (int)(gridDim.x >> 3) / G;        // row streams per XCD group
    if (kk >= spx * G) return;                         // no part of any stream (uniform)
    const int p = kk % G;
    const int q = (kk / G) * 8 + x;
    const int S = spx * 8;
    if (q >= R) return;
    const int ntile = (R - q + S - 1) / S;             // this stream's rows: positions q, q + S, ...
    const int pbase = p * ROW_PART;

    const lds_ptr<unsigned> s_bits = lds_at<unsigned>(RC_S_BITS);
    const lds_ptr<int> s_ring = lds_at<int>(RC_S_RING);
    const lds_ptr<float> stage = lds_at<float>(ROW_STAGE);   // [2][ROW_PART]

    RowcLane n;
    rowc_load(a, p, tid, n);
#pragma unroll
    for (int s = 0; s < 64; ++s) __asm__ volatile("" : "+v"(n.w[s]));   // keep resident
#pragma unroll
    for (int s = 0; s < 32; ++s) __asm__ volatile("" : "+v"(n.o[s]));

    const int ncopy = CW / 256;                        // 1 KB copies per chunk
    const int mycopies = wave < ncopy ? (ncopy - wave + RC_WAVES - 1) / RC_WAVES : 0;
    auto pos_row = [&](int i) -> int { return a.row_base + q + i * S; };   // identity work list
    auto prefetch = [&](int i) {
        if (a.list_in && wave == 0 && lane == 0) row_copy4(a.list_in + q + i * S, RC_S_RING + 4u * (uint32_t)(i % 3));
    };
    auto ring_row = [&](int i) -> int {
        return a.list_in ? __builtin_amdgcn_readfirstlane(s_ring[i % 3]) : pos_row(i);
    };
    // this wave's k-th copy of a chunk (global address chunk_src) into the buffer at
    // byte `buf`.  The G parts of a row run on one XCD and stage the same chunk at
    // about the same time; each starts at its own share of the chunk's 1 KB pieces
    // (part p at piece p * ncopy / G), so they do not all ask the same L2 lines at
    // once (C4 forward 23.5 -> 20.8 ms)
    const uint64_t ybase = uniform_ptr(a.yin);
    const int rot = (int)(((int64_t)p * ncopy) / G);
    auto copy = [&](uint64_t chunk_src, uint32_t buf, int k) {
        int cc = wave + k * RC_WAVES;
        if (cc >= ncopy) return;
        cc += rot;
        if (cc >= ncopy) cc -= ncopy;
        row_copy16(chunk_src + 1024ull * (uint32_t)cc, 16u * (uint32_t)lane, buf + 1024u * (uint32_t)cc);
    };
    auto chunk_src = [&](int row, int c) -> uint64_t {
        uint64_t s = ybase + 4ull * ((uint64_t)(uint32_t)row * (uint64_t)N + (uint64_t)(c * CW));
        __asm__ volatile("" : "+s"(s));
        return s;
    };

    // wave 0's liveness pipeline (as in the one-row-tile kernel)
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
    // the previous row's outputs: the part's slice as 16-byte stores
    auto store_stage = [&](int row, int sbuf) {
        const int e = 4 * tid;
        if (e < ROW_PART) {
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
    __syncthreads();                                   // the overflow list and the row ids have landed
    int row_c = ring_row(0);
    {
        const uint64_t cs = chunk_src(row_c, 0);
        for (int k = 0; k < mycopies; ++k) copy(cs, 0u, k);
    }
    int row_p = 0;
    for (int i = 0; i < ntile; ++i) {
        const bool more = i + 1 < ntile;
        int row_n = 0;
        float acca = 0.f, accb = 0.f;
        auto step = [&](auto cc) {
            constexpr int CH = decltype(cc)::value;
            uint32_t buf = (uint32_t)(CH & 1) * ROW_BUF_BYTES;
            __asm__ volatile("" : "+s"(buf));
            __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");   // this wave's copies of the chunk have landed
            __syncthreads();                                        // everyone's have; the other buffer is free
            if constexpr (CH == 0) {
                if (i > 0) {
                    if (wave == 0) {
                        const unsigned bit = s_bits[(i - 1) & 1];
                        advance(q + (i - 1) * S, row_p, bit);       // before any store: nothing outstanding
                        if (lane == 0) s_bits[(i - 1) & 1] = 0u;
                    }
                    store_stage(row_p, (i - 1) & 1);
                }
                row_n = more ? ring_row(i + 1) : 0;
                if (i + 2 < ntile) prefetch(i + 2);
            }
            // the next chunk step's copies: chunk CH + 1 of this row, or chunk 0 of the
            // next row, all issued before the first compute group (a whole chunk step
            // to land; spreading them over the groups was 8 % slower per layer)
            const bool next = CH + 1 < C || more;
            const uint64_t nsrc = chunk_src(CH + 1 < C ? row_c : row_n, CH + 1 < C ? CH + 1 : 0);
            const uint32_t nbuf = (uint32_t)((CH + 1) & 1) * ROW_BUF_BYTES;
            int myc = next ? mycopies : 0;
            __asm__ volatile("" : "+s"(myc));
            auto hook = [&](int g) {
                if (g == 0)
                    for (int k = 0; k < myc; ++k) copy(nsrc, nbuf, k);
            };
            rowc_chunk<C, CH, RS>(n, buf, acca, accb, hook);
        };
        step(std::integral_constant<int, 0>{});
        step(std::integral_constant<int, 1>{});
        if constexpr (C == 4) {
            step(std::integral_constant<int, 2>{});
            step(std::integral_constant<int, 3>{});
        }
        const float ya = fminf(fmaxf(acca + n.ba, 0.f), a.clamp);
        const float yb = fminf(fmaxf(accb + n.bb, 0.f), a.clamp);
        const lds_ptr<float> st = stage + (i & 1) * ROW_PART;
        st[n.jab & 0xffffu] = ya;
        st[n.jab >> 16] = yb;
        const bool nz = ya != 0.f || yb != 0.f;
        if (__ballot(nz) != 0ull && lane == 0)
            __hip_atomic_fetch_or(s_bits + (i & 1), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        row_p = row_c;
        row_c = row_n;
    }
    // drain: the last row's outputs and the rest of the liveness pipeline
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

// the lane images of layer l within the stacked tables
__device__ __forceinline__ void rowc_layer_tables(const ChainArgs& c, int l, LayerArgs& a) {
    const size_t parts = (size_t)c.row_parts;
    a.rowc_img = c.rowc_img + (size_t)l * parts * ROWC_IMG * ROW_NT;
    a.rowc_meta = c.rowc_meta + (size_t)l * parts * ROW_NT * 4;
    a.rowc_ovf = c.rowc_ovf + (size_t)l * parts * ROWC_OVF_CAP * 2;
}

template <int C>
__global__ __launch_bounds__(ROW_NT) void k_layer_rowc(LayerArgs a) {
    run_layer_rowc<C, 2>(a, a.cnt_in ? *a.cnt_in : a.nrows);   // (4: 10.56 against 10.36 ms per C4 layer)
}

template <int C>
__global__ __launch_bounds__(ROW_NT) void k_chain_rowc(ChainArgs) {
    int* s_ok = (int*)lds_at<int>(RC_S_OK);
    unsigned gen = 0u;
    for (int l = 0;; ++l) {
        {
            const ChainArgs c = reload_chain_args();
            if (l >= c.L) break;
            const int R = (l == 0 || !c.compaction) ? c.rows : ld_count(&c.cnt[l]);
            if (R == 0) break;
            LayerArgs a = chain_layer_args(c, l, R);
            a.row_parts = c.row_parts;
            a.row_words = c.row_words;
            rowc_layer_tables(c, l, a);
            run_layer_rowc<C, 2>(a, R);                  // (4: C4 forward 23.0 against 20.6 ms)
        }
        const ChainArgs c = reload_chain_args();
        if (!grid_barrier(c.bar, gen, c.err, s_ok)) return;
    }
}

template __global__ void k_layer_rowc<2>(LayerArgs);
template __global__ void k_layer_rowc<4>(LayerArgs);
template __global__ void k_chain_rowc<2>(ChainArgs);
template __global__ void k_chain_rowc<4>(ChainArgs);

// ---------------------------------------------------------------- uniform-weight two-part kernel
// For nets whose layers each carry one weight value w (the sparse-DNN challenge's
// nets have one weight for every connection), the register positions need no
// weights: a lane holds the offsets of two pairs, pair l of sub-parts 2p and 2p + 1
// of the chunked kernel's lane images, so a workgroup computes 4096 neurons and each
// row is staged from L2 once per 4096 neurons instead of once per 2048 (the staging
// is what bounds the chunked kernel at 65536 neurons).  What differs from it:
//  * padding positions read zero words: the last RU_ZERO ids (128 bytes) of every
//    staged chunk go to a side slot instead of the buffer, so the buffer ends in 32
//    zero words, one in each LDS bank; the builder makes every slot on those ids an
//    overflow entry, and k_rowu_pads points each padding offset at the zero word of
//    the bank the create-time order gave it (with 4 zero words, so 4 banks for all
//    padding, the two-layer C4 forward took 17.3 ms against 16.8);
//  * overflow entries are 4 bytes (offset | owner << 16 | side << 17), the lists of
//    both sub-parts (at most RU_OVF_CAP entries each) in the LDS one part's 8-byte
//    list takes;
//  * one output stage of 4096 floats: it is written after the last chunk step of a
//    row and read after the first barrier of the next one, C - 1 >= 1 barriers later.
// Every neuron sums its slots in the images' order with fused multiply-adds by w, as
// the chunked kernel does with the same images (padding adds w * 0 here and 0 * y
// there), so the two give equal outputs.
namespace {

constexpr uint32_t RU_SIDE = (uint32_t)LDS_BYTES - 2u * 4u * RU_ZERO;   // [2][RU_ZERO floats], one per buffer
constexpr uint32_t RU_OVF_HALF = (uint32_t)RU_OVF_CAP * 4u;              // one sub-part's 4-byte entries

struct RowuPair {
    uint32_t o[32];    // 64 positions: 16-bit LDS byte offsets within the chunk buffer
    uint32_t split;    // byte c: positions of neuron A in chunk c (B's follow)
    uint32_t ocnt;     // byte c: overflow entries of chunk c
    uint32_t obase;    // LDS byte address of the pair's first overflow entry
    uint32_t jab;      // neurons A (low 16 bits) and B (high) within the sub-part
    float ba, bb;
};

// Pair `tid` of sub-part sp (0 or 1) of the workgroup, image part `ip`; the
// sub-part's overflow list goes to LDS with the side bit set on entries of a chunk's
// last RU_ZERO ids.
__device__ __forceinline__ void rowu_load(const LayerArgs& a, int ip, int sp, int tid, int CW, RowuPair& n) {
    const uint32_t* img = a.rowc_img + (size_t)ip * ROWC_IMG * ROW_NT + tid;
#pragma unroll
    for (int r = 0; r < 32; ++r) n.o[r] = img[(size_t)(64 + r) * ROW_NT];
    const uint4 m = reinterpret_cast<const uint4*>(a.rowc_meta)[(size_t)ip * ROW_NT + tid];
    n.jab = m.x;
    n.split = m.y;
    n.ocnt = m.z;
    n.obase = ROWC_OVF + (uint32_t)sp * RU_OVF_HALF + 4u * m.w;
    n.ba = a.b[ip * ROW_PART + (int)(m.x & 0xffffu)];
    n.bb = a.b[ip * ROW_PART + (int)(m.x >> 16)];
    const uint2* src = reinterpret_cast<const uint2*>(a.rowc_ovf + (size_t)ip * ROWC_OVF_CAP * 2);
    const uint32_t last = 4u * (uint32_t)(CW - RU_ZERO);
    for (int e = tid; e < RU_OVF_CAP; e += ROW_NT) {
        const uint32_t y = src[e].y;
        *lds_at<uint32_t>(ROWC_OVF + (uint32_t)sp * RU_OVF_HALF + 4u * (uint32_t)e) =
            y | ((y & 0xffffu) >= last ? (1u << 17) : 0u);
    }
}

__device__ __forceinline__ uint32_t rowu_addr(const RowuPair& n, int P, uint32_t buf) {
    return __builtin_amdgcn_perm(buf, n.o[P >> 1], (P & 1) ? 0x07060302u : 0x07060100u);
}

template <int C, int CH, int RS, int G>
__device__ __forceinline__ void rowu_reads(const RowuPair& n, uint32_t buf, float (&r)[RS]) {
    constexpr int PC = 64 / C;
#pragma unroll
    for (int u = 0; u < RS; ++u) r[u] = row_lds_read(rowu_addr(n, PC * CH + RS * G + u, buf));
}

template <int RS, int G>
__device__ __forceinline__ void rowu_fmas(float wu, uint32_t splitc, const float (&r)[RS], float& cur, float& acca,
                                          float& accb) {
#pragma unroll
    for (int u = 0; u < RS; ++u) {
        const int k = RS * G + u;
        const bool sw = (uint32_t)k == splitc;
        acca = sw ? cur : acca;
        cur = sw ? accb : cur;
        cur = fmaf(wu, r[u], cur);
    }
    __asm__ volatile("" : "+v"(cur), "+v"(acca), "+v"(accb) : : "memory");
}

template <int C, int CH, int RS, int G, typename Hook>
__device__ __forceinline__ void rowu_group(const RowuPair& n, float wu, uint32_t buf, uint32_t splitc, float& cur,
                                           float& acca, float& accb, float (&v)[2][RS], Hook& hook) {
    constexpr int PC = 64 / C;
    hook(G);
    if constexpr (G + 1 < PC / RS) rowu_reads<C, CH, RS, G + 1>(n, buf, v[(G + 1) & 1]);
    rowu_fmas<RS, G>(wu, splitc, v[G & 1], cur, acca, accb);
    if constexpr (G + 1 < PC / RS) rowu_group<C, CH, RS, G + 1>(n, wu, buf, splitc, cur, acca, accb, v, hook);
}

// Chunk CH of the row (buffer at `buf`) for one pair: its positions.
template <int C, int CH, int RS, typename Hook>
__device__ __forceinline__ void rowu_positions(const RowuPair& n, float wu, uint32_t buf, float& acca, float& accb,
                                               Hook&& hook) {
    constexpr int PC = 64 / C;
    uint32_t splitc = byte_of(n.split, CH);
    __asm__ volatile("" : "+v"(splitc));
    float cur = acca;
    float v[2][RS];
    rowu_reads<C, CH, RS, 0>(n, buf, v[0]);
    rowu_group<C, CH, RS, 0>(n, wu, buf, splitc, cur, acca, accb, v, hook);
    const bool none = splitc == (uint32_t)PC;
    acca = none ? cur : acca;
    accb = none ? accb : cur;
}

// LDS byte address of the pair's first overflow entry of chunk CH.
template <int CH>
__device__ __forceinline__ uint32_t rowu_first_entry(const RowuPair& n) {
    uint32_t ea = n.obase;
#pragma unroll
    for (int c = 0; c < CH; ++c) ea += 4u * byte_of(n.ocnt, c);
    return ea;
}

// The overflow entries of chunk CH of both pairs, one entry of each per pass (two
// independent chains of dependent LDS reads instead of one after the other; each
// pair's entries still in their order).  en0 / en1: the first entries, read by the
// caller ahead (a lane without one read a word it does not use).
template <int CH>
__device__ __forceinline__ void rowu_overflow(const RowuPair& n0, const RowuPair& n1, float wu, uint32_t buf,
                                              uint32_t side, uint32_t ea0, uint32_t ea1, uint32_t en0, uint32_t en1,
                                              float& acca0, float& accb0, float& acca1, float& accb1) {
    const int cnt0 = (int)byte_of(n0.ocnt, CH), cnt1 = (int)byte_of(n1.ocnt, CH);
    const int cmax = max(cnt0, cnt1);
    auto addr = [&](uint32_t en) {
        const uint32_t off = en & 0xffffu;
        return (en >> 17) ? side + (off & (4u * RU_ZERO - 1u)) : (buf | off);
    };
    for (int e = 0; e < cmax; ++e) {
        const float x0 = row_lds_read(addr(en0));
        const float x1 = row_lds_read(addr(en1));
        if (e < cnt0) {
            if ((en0 >> 16) & 1u)
                accb0 = fmaf(wu, x0, accb0);
            else
                acca0 = fmaf(wu, x0, acca0);
        }
        if (e < cnt1) {
            if ((en1 >> 16) & 1u)
                accb1 = fmaf(wu, x1, accb1);
            else
                acca1 = fmaf(wu, x1, acca1);
        }
        // the next entries (a lane past its count reads its last one again)
        en0 = *lds_at<uint32_t>(ea0 + 4u * (uint32_t)min(e + 1, max(cnt0 - 1, 0)));
        en1 = *lds_at<uint32_t>(ea1 + 4u * (uint32_t)min(e + 1, max(cnt1 - 1, 0)));
    }
}

}  // namespace

template <int C, int RS>
__device__ __forceinline__ void run_layer_rowu(const LayerArgs& a, int R) {
    const int N = a.N;
    const int CW = N / C;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int G = a.row_parts / 2;                     // parts of 2 ROW_PART neurons (the host keeps row_parts even)
    if (G < 1) return;
    const int b = blockIdx.x, x = b & 7, kk = b >> 3;
    const int spx = (int)(gridDim.x >> 3) / G;        // row streams per XCD group
    if (kk >= spx * G) return;                         // no part of any stream (uniform)
    const int p = kk % G;
    const int q = (kk / G) * 8 + x;
    const int S = spx * 8;
    if (q >= R) return;
    const int ntile = (R - q + S - 1) / S;             // this stream's rows: positions q, q + S, ...
    const int pbase = p * 2 * ROW_PART;

    const lds_ptr<unsigned> s_bits = lds_at<unsigned>(RC_S_BITS);
    const lds_ptr<int> s_ring = lds_at<int>(RC_S_RING);
    const lds_ptr<float> stage = lds_at<float>(ROW_STAGE);   // [2 ROW_PART], one stage

    // the layer's weight (every weight of the layer has this value)
    const float wu = __uint_as_float((uint32_t)__builtin_amdgcn_readfirstlane((int)__float_as_uint(a.w[0])));
    RowuPair n0, n1;
    rowu_load(a, 2 * p, 0, tid, CW, n0);
    rowu_load(a, 2 * p + 1, 1, tid, CW, n1);
#pragma unroll
    for (int s = 0; s < 32; ++s) __asm__ volatile("" : "+v"(n0.o[s]), "+v"(n1.o[s]));   // keep resident
    // the zero words: the last RU_ZERO words of both buffers, which no copy writes
    if (tid < 2 * RU_ZERO)
        *lds_at<float>((uint32_t)(tid / RU_ZERO) * ROW_BUF_BYTES + 4u * (uint32_t)(CW - RU_ZERO + tid % RU_ZERO)) = 0.f;

    // a chunk's 1 KB pieces: all but the last as plain copies spread over the waves,
    // the last one (its last 128 bytes, lanes 56..63, to the buffer's side slot) by
    // the wave left with one copy fewer, before its compute (control flow among the
    // plain copies, which run between the compute groups, cost 0.7 ms per C4 layer)
    const int ncopy = CW / 256;
    const int nplain = ncopy - 1;
    const int mycopies = wave < nplain ? (nplain - wave + RC_WAVES - 1) / RC_WAVES : 0;
    const int lastw = nplain % RC_WAVES;
    auto pos_row = [&](int i) -> int { return a.row_base + q + i * S; };   // identity work list
    auto prefetch = [&](int i) {
        if (a.list_in && wave == 0 && lane == 0) row_copy4(a.list_in + q + i * S, RC_S_RING + 4u * (uint32_t)(i % 3));
    };
    auto ring_row = [&](int i) -> int {
        return a.list_in ? __builtin_amdgcn_readfirstlane(s_ring[i % 3]) : pos_row(i);
    };
    const uint64_t ybase = uniform_ptr(a.yin);
    const int rot = (int)(((int64_t)p * nplain) / G);
    // this wave's k-th plain copy of a chunk into the buffer at byte `buf`
    auto copy = [&](uint64_t chunk_src, uint32_t buf, int k) {
        int cc = wave + k * RC_WAVES;
        if (cc >= nplain) return;
        cc += rot;
        if (cc >= nplain) cc -= nplain;
        row_copy16(chunk_src + 1024ull * (uint32_t)cc, 16u * (uint32_t)lane, buf + 1024u * (uint32_t)cc);
    };
    auto copy_last = [&](uint64_t chunk_src, uint32_t buf, uint32_t side) {
        constexpr int L0 = 64 - RU_ZERO / 4;               // first lane of the displaced bytes
        const uint64_t src = chunk_src + 1024ull * (uint32_t)nplain;
        if (lane < L0)
            row_copy16(src, 16u * (uint32_t)lane, buf + 1024u * (uint32_t)nplain);
        else
            row_copy16(src, 16u * (uint32_t)lane, side - 16u * (uint32_t)L0);   // lands at `side`
    };
    auto chunk_src = [&](int row, int c) -> uint64_t {
        uint64_t s = ybase + 4ull * ((uint64_t)(uint32_t)row * (uint64_t)N + (uint64_t)(c * CW));
        __asm__ volatile("" : "+s"(s));
        return s;
    };

    // wave 0's liveness pipeline (as in the one-row-tile kernel)
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
    // the previous row's outputs: the part's 4096 floats as 16-byte stores
    auto store_stage = [&](int row) {
        const int e = 4 * tid;
        const lds_ptr<const float> sp = lds_at<const float>(ROW_STAGE + 4u * (uint32_t)e);
        const float4 v = make_float4(sp[0], sp[1], sp[2], sp[3]);
        const size_t o = (size_t)row * N + pbase + e;
        *reinterpret_cast<float4*>(a.yout + o) = v;
        if (a.ycopy) *reinterpret_cast<float4*>(a.ycopy + o) = v;
    };

    if (tid == 0) { s_bits[0] = 0u; s_bits[1] = 0u; }
    prefetch(0);
    if (ntile > 1) prefetch(1);
    __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
    __syncthreads();                                   // overflow lists, zero words and row ids are in place
    int row_c = ring_row(0);
    {
        const uint64_t cs = chunk_src(row_c, 0);
        for (int k = 0; k < mycopies; ++k) copy(cs, 0u, k);
        if (wave == lastw) copy_last(cs, 0u, RU_SIDE);
    }
    int row_p = 0;
    for (int i = 0; i < ntile; ++i) {
        const bool more = i + 1 < ntile;
        int row_n = 0;
        float acca0 = 0.f, accb0 = 0.f, acca1 = 0.f, accb1 = 0.f;
        auto step = [&](auto cc) {
            constexpr int CH = decltype(cc)::value;
            uint32_t buf = (uint32_t)(CH & 1) * ROW_BUF_BYTES;
            __asm__ volatile("" : "+s"(buf));
            const uint32_t side = RU_SIDE + 4u * RU_ZERO * (uint32_t)(CH & 1);
            __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");   // this wave's copies of the chunk have landed
            __syncthreads();                                        // everyone's have; the other buffer is free
            if constexpr (CH == 0) {
                if (i > 0) {
                    if (wave == 0) {
                        const unsigned bit = s_bits[(i - 1) & 1];
                        advance(q + (i - 1) * S, row_p, bit);       // before any store: nothing outstanding
                        if (lane == 0) s_bits[(i - 1) & 1] = 0u;
                    }
                    store_stage(row_p);
                }
                row_n = more ? ring_row(i + 1) : 0;
                if (i + 2 < ntile) prefetch(i + 2);
            }
            // the next chunk step's copies, all issued before the first compute group
            const bool next = CH + 1 < C || more;
            const uint64_t nsrc = chunk_src(CH + 1 < C ? row_c : row_n, CH + 1 < C ? CH + 1 : 0);
            const uint32_t nbuf = (uint32_t)((CH + 1) & 1) * ROW_BUF_BYTES;
            const uint32_t nside = RU_SIDE + 4u * RU_ZERO * (uint32_t)((CH + 1) & 1);
            int myc = next ? mycopies : 0;
            __asm__ volatile("" : "+s"(myc));
            if (next && wave == lastw) copy_last(nsrc, nbuf, nside);
            auto hook = [&](int g) {
                if (g == 0)
                    for (int k = 0; k < myc; ++k) copy(nsrc, nbuf, k);
            };
            auto nohook = [](int) {};
            const uint32_t ea0 = rowu_first_entry<CH>(n0), ea1 = rowu_first_entry<CH>(n1);
            rowu_positions<C, CH, RS>(n0, wu, buf, acca0, accb0, hook);
            // the first overflow entries, read while the second pair's positions run
            const uint32_t en0 = *lds_at<uint32_t>(ea0), en1 = *lds_at<uint32_t>(ea1);
            rowu_positions<C, CH, RS>(n1, wu, buf, acca1, accb1, nohook);
            rowu_overflow<CH>(n0, n1, wu, buf, side, ea0, ea1, en0, en1, acca0, accb0, acca1, accb1);
        };
        step(std::integral_constant<int, 0>{});
        step(std::integral_constant<int, 1>{});
        if constexpr (C == 4) {
            step(std::integral_constant<int, 2>{});
            step(std::integral_constant<int, 3>{});
        }
        const float ya0 = fminf(fmaxf(acca0 + n0.ba, 0.f), a.clamp);
        const float yb0 = fminf(fmaxf(accb0 + n0.bb, 0.f), a.clamp);
        const float ya1 = fminf(fmaxf(acca1 + n1.ba, 0.f), a.clamp);
        const float yb1 = fminf(fmaxf(accb1 + n1.bb, 0.f), a.clamp);
        stage[n0.jab & 0xffffu] = ya0;
        stage[n0.jab >> 16] = yb0;
        stage[ROW_PART + (n1.jab & 0xffffu)] = ya1;
        stage[ROW_PART + (n1.jab >> 16)] = yb1;
        const bool nz = ya0 != 0.f || yb0 != 0.f || ya1 != 0.f || yb1 != 0.f;
        if (__ballot(nz) != 0ull && lane == 0)
            __hip_atomic_fetch_or(s_bits + (i & 1), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        row_p = row_c;
        row_c = row_n;
    }
    // drain: the last row's outputs and the rest of the liveness pipeline
    __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
    __syncthreads();
    if (wave == 0) {
        advance(q + (ntile - 1) * S, row_p, s_bits[(ntile - 1) & 1]);
        __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
        advance(-1, 0, 0u);
        __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
        advance(-1, 0, 0u);
    }
    store_stage(row_p);
    __asm__ volatile("s_waitcnt vmcnt(0)" : : : "memory");
    __syncthreads();                                   // the LDS is reused by the next layer
}

template <int C>
__global__ __launch_bounds__(ROW_NT) void k_layer_rowu(LayerArgs a) {
    run_layer_rowu<C, 2>(a, a.cnt_in ? *a.cnt_in : a.nrows);
}

template <int C>
__global__ __launch_bounds__(ROW_NT) void k_chain_rowu(ChainArgs) {
    int* s_ok = (int*)lds_at<int>(RC_S_OK);
    unsigned gen = 0u;
    for (int l = 0;; ++l) {
        {
            const ChainArgs c = reload_chain_args();
            if (l >= c.L) break;
            const int R = (l == 0 || !c.compaction) ? c.rows : ld_count(&c.cnt[l]);
            if (R == 0) break;
            LayerArgs a = chain_layer_args(c, l, R);
            a.row_parts = c.row_parts;
            a.row_words = c.row_words;
            rowc_layer_tables(c, l, a);
            run_layer_rowu<C, 2>(a, R);
        }
        const ChainArgs c = reload_chain_args();
        if (!grid_barrier(c.bar, gen, c.err, s_ok)) return;
    }
}

template __global__ void k_layer_rowu<2>(LayerArgs);
template __global__ void k_layer_rowu<4>(LayerArgs);
template __global__ void k_chain_rowu<2>(ChainArgs);
template __global__ void k_chain_rowu<4>(ChainArgs);

// Points every padding position (weight 0) of the lane images at the zero word of
// its LDS bank among the uniform-weight kernel's RU_ZERO zero words, which start at
// byte `zbase` of the chunk buffer (the chunked kernel multiplies padding by 0
// wherever it points).  One thread per lane image.
__global__ void k_rowu_pads(uint32_t* img, int64_t lanes, uint32_t zbase) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < lanes; t += (int64_t)gridDim.x * blockDim.x) {
        uint32_t* im = img + (t / ROW_NT) * (int64_t)ROWC_IMG * ROW_NT + t % ROW_NT;
        auto zero_word = [&](uint32_t off) { return zbase + 4u * ((off >> 2) & (RU_ZERO - 1u)); };
        for (int r = 0; r < 32; ++r) {
            uint32_t o = im[(size_t)(64 + r) * ROW_NT];
            if ((im[(size_t)(2 * r) * ROW_NT] & 0x7fffffffu) == 0u) o = (o & 0xffff0000u) | zero_word(o & 0xffffu);
            if ((im[(size_t)(2 * r + 1) * ROW_NT] & 0x7fffffffu) == 0u) o = (o & 0xffffu) | (zero_word(o >> 16) << 16);
            im[(size_t)(64 + r) * ROW_NT] = o;
        }
    }
}

// flags[l] = 1 where some weight of layer l differs (bitwise) from the layer's first.
__global__ void k_weights_uniform(const float* w, int64_t per_layer, int64_t total, int32_t* flags) {
    const uint32_t* wb = reinterpret_cast<const uint32_t*>(w);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = i / per_layer;
        if (wb[i] != wb[l * per_layer]) flags[l] = 1;
    }
}

// Per-neuron slot counts per chunk (byte c) of `neurons` consecutive neurons of N
// inputs each (several layers stacked): the host pairs neurons from them.
__global__ void k_rowc_counts(const int32_t* idx, int64_t neurons, int32_t N, int32_t C, uint32_t* counts) {
    const int CW = N / C;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < neurons; j += (int64_t)gridDim.x * blockDim.x) {
        uint32_t cnt = 0u;
        for (int k = 0; k < K; ++k) {
            const int id = idx[j * K + k];
            const int c = id / CW;
            cnt += 1u << (8 * (c < C ? c : C - 1));
        }
        counts[j] = cnt;
    }
}

// The lane images of one (part, layer) = (blockIdx.x, blockIdx.y), one thread per
// pair (lane): positions per chunk (A's slots, then B's, then weight-0 padding),
// the pair words and the part's overflow list, entries of a lane in chunk order
// (A's excess, then B's) and lanes in order.  Slots on a chunk's last `disp` ids
// (0, or RU_ZERO for the uniform-weight kernel, which keeps those bytes of a staged
// chunk outside the buffer and zero words in their place) are always overflow
// entries.  A list longer than ROWC_OVF_CAP keeps only what fits, a lane whose
// entries do not all fit keeps none, and status[0] is set to 1 (the host then does
// not use the images); status[1] becomes the longest list's length.
__global__ __launch_bounds__(ROW_NT) void k_rowc_build(const int32_t* idx, const float* w, const uint32_t* pairs,
                                                       int32_t N, int32_t C, int32_t disp, uint32_t* img,
                                                       uint32_t* meta, uint32_t* ovf, int32_t* status) {
    __shared__ int s_tot[RC_WAVES];
    const int p = blockIdx.x, l = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int parts = gridDim.x;
    const int CW = N / C, PC = 64 / C;
    const uint32_t pr = pairs[(size_t)l * (N / 2) + (size_t)p * ROW_NT + tid];
    const int j[2] = {p * ROW_PART + (int)(pr & 0xffffu), p * ROW_PART + (int)(pr >> 16)};
    const int32_t* ids[2] = {idx + ((size_t)l * N + j[0]) * K, idx + ((size_t)l * N + j[1]) * K};
    const float* ws[2] = {w + ((size_t)l * N + j[0]) * K, w + ((size_t)l * N + j[1]) * K};
    // slots per chunk, and those that may take a position (not on the chunk's last 4 ids)
    int cnt[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, cntp[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
    for (int h = 0; h < 2; ++h)
        for (int k = 0; k < K; ++k) {
            const int id = max(ids[h][k], 0);
            const int c = min(id / CW, C - 1);
            cnt[h][c] += 1;
            cntp[h][c] += (id - c * CW < CW - disp) ? 1 : 0;
        }
    uint32_t split = 0u, ocnt = 0u;
    int tot = 0;
    int m[4] = {0, 0, 0, 0};
    for (int c = 0; c < C; ++c) {
        m[c] = min(cntp[0][c], PC);
        const int ova = cnt[0][c] - m[c];
        const int ovb = cnt[1][c] - min(cntp[1][c], PC - m[c]);
        split |= (uint32_t)m[c] << (8 * c);
        ocnt |= (uint32_t)(ova + ovb) << (8 * c);
        tot += ova + ovb;
    }
    // lanes' first entries: exclusive scan over the workgroup
    int v = tot;
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off);
        if (lane >= off) v += t;
    }
    if (lane == 63) s_tot[wave] = v;
    __syncthreads();
    int base = v - tot;
    for (int x = 0; x < wave; ++x) base += s_tot[x];
    const bool fits = base + tot <= ROWC_OVF_CAP;
    if (!fits) atomicOr(status, 1);
    if (tid == ROW_NT - 1) atomicMax(status + 1, base + tot);   // the last lane's end: the list's length
    const size_t pl = (size_t)l * parts + p;
    uint32_t* im = img + pl * ROWC_IMG * ROW_NT + tid;
    uint32_t* ov = ovf + pl * ROWC_OVF_CAP * 2;
    float wpos[64];
    uint32_t opos[64];
    for (int r = 0; r < 64; ++r) {
        wpos[r] = 0.f;
        opos[r] = 0u;
    }
    // each neuron's slots of a chunk in ascending order; A's from the chunk's first
    // position, B's after A's; the rest of each chunk's slots are overflow entries
    int e = base;
    for (int c = 0; c < C; ++c)
        for (int h = 0; h < 2; ++h) {
            const int first = h == 0 ? 0 : m[c];
            const int room = h == 0 ? m[c] : PC - m[c];
            int rank = 0;
            for (int k = 0; k < K; ++k) {
                const int id = ids[h][k];
                if (min(max(id, 0) / CW, C - 1) != c) continue;
                const uint32_t off = (4u * (uint32_t)(id - c * CW)) & 0xffffu;
                if (id - c * CW < CW - disp && rank < room) {
                    wpos[c * PC + first + rank] = ws[h][k];
                    opos[c * PC + first + rank] = off;
                    ++rank;
                } else {
                    if (fits) {
                        ov[2 * e] = __float_as_uint(ws[h][k]);
                        ov[2 * e + 1] = off | ((uint32_t)h << 16);
                    }
                    ++e;
                }
            }
        }
    for (int r = 0; r < 64; ++r) im[(size_t)r * ROW_NT] = __float_as_uint(wpos[r]);
    for (int r = 0; r < 32; ++r) im[(size_t)(64 + r) * ROW_NT] = opos[2 * r] | (opos[2 * r + 1] << 16);
    reinterpret_cast<uint4*>(meta)[pl * ROW_NT + tid] = make_uint4(pr, split, fits ? ocnt : 0u, (uint32_t)base);
}

// Bank order of the lane images: for one (layer, part, half-wave block of 32
// lanes, chunk) per thread, the positions of the chunk are reordered so that at
// each position the block's 32 lanes read few LDS banks twice (a 4-byte LDS read
// is served per half-wave, bank = word address mod 32; in ascending order the 32
// reads of a position hit random banks, about 3.5 passes per read).  A lane's
// items are its A slots, its B slots and its padding (weight 0, which adds nothing
// wherever it sits, so a zero-weight slot counts as padding too); B's slots may
// only follow all of A's, so the lane's switch position becomes its first step
// with a B slot.  Greedy per step: lanes with the fewest candidate banks choose
// first, each the least-loaded bank among its candidates (padding may take any
// bank, at a word of that bank).  Each neuron then sums its chunk's slots in this
// fixed order, so results stay deterministic (they differ from ascending order
// only by rounding).
__global__ void k_rowc_sched(uint32_t* img, uint32_t* meta, int64_t tasks, int32_t C) {
    const int PC = 64 / C;
    // one thread per (layer, part, block) = task, its chunks in turn: the chunks of a
    // block share the lanes' split words
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tasks; t += (int64_t)gridDim.x * blockDim.x) {
        const int blk = (int)(t % 32);
        const int64_t lp = t / 32;
        uint32_t* im = img + lp * ROWC_IMG * ROW_NT + blk * 32;
        uint32_t* me = meta + ((size_t)lp * ROW_NT + blk * 32) * 4;
        for (int c = 0; c < C; ++c) {
        // per lane: items (A's real slots, then B's) as (bank, source position); the
        // choice per step: a source position, or 0x80 | bank for padding
        uint8_t bank[32][32], srcp[32][32], outp[32][32];
        int na[32], nb[32], npad[32], ra[32], rb[32], split[32];
        uint32_t taken[32];
        for (int l = 0; l < 32; ++l) {
            const int m = (int)byte_of(me[4 * l + 1], c);
            na[l] = nb[l] = 0;
            for (int pass = 0; pass < 2; ++pass)
                for (int k = pass ? m : 0; k < (pass ? PC : m); ++k) {
                    const int pos = c * PC + k;
                    const uint32_t w = im[(size_t)pos * ROW_NT + l];
                    if ((w & 0x7fffffffu) == 0u) continue;             // padding or a zero weight
                    const uint32_t ow = im[(size_t)(64 + pos / 2) * ROW_NT + l];
                    const uint32_t off = (pos & 1) ? (ow >> 16) : (ow & 0xffffu);
                    const int it = na[l] + nb[l];
                    bank[l][it] = (uint8_t)((off >> 2) & 31u);
                    srcp[l][it] = (uint8_t)k;
                    if (pass) ++nb[l]; else ++na[l];
                }
            npad[l] = PC - na[l] - nb[l];
            ra[l] = na[l];
            rb[l] = nb[l];
            split[l] = PC;
            taken[l] = 0u;
        }
        for (int st = 0; st < PC; ++st) {
            int load[32];
            for (int q = 0; q < 32; ++q) load[q] = 0;
            uint32_t cand[32];
            int order[32], ncand[32];
            for (int l = 0; l < 32; ++l) {
                uint32_t mk = 0u;
                const int b0 = ra[l] > 0 ? 0 : na[l], n = ra[l] > 0 ? na[l] : nb[l];
                for (int i = 0; i < n; ++i)
                    if (!((taken[l] >> (b0 + i)) & 1u)) mk |= 1u << bank[l][b0 + i];
                cand[l] = mk;
                ncand[l] = npad[l] > 0 ? 33 : __popc(mk);
                order[l] = l;
            }
            for (int i = 1; i < 32; ++i)   // fewest candidates first (insertion sort, stable)
                for (int j = i; j > 0 && ncand[order[j]] < ncand[order[j - 1]]; --j) {
                    const int x = order[j];
                    order[j] = order[j - 1];
                    order[j - 1] = x;
                }
            for (int oi = 0; oi < 32; ++oi) {
                const int l = order[oi];
                int best = -1, bl = 1 << 30;
                for (int q = 0; q < 32; ++q)
                    if (((cand[l] >> q) & 1u) && load[q] < bl) { bl = load[q]; best = q; }
                int pb = -1, pl = 1 << 30;
                if (npad[l] > 0)
                    for (int q = 0; q < 32; ++q)
                        if (load[q] < pl) { pl = load[q]; pb = q; }
                if (best < 0 || (pb >= 0 && pl < bl)) {        // padding on a freer bank
                    outp[l][st] = (uint8_t)(0x80u | (uint32_t)pb);
                    --npad[l];
                    ++load[pb];
                    continue;
                }
                const bool inA = ra[l] > 0;
                const int b0 = inA ? 0 : na[l], n = inA ? na[l] : nb[l];
                for (int i = 0; i < n; ++i) {
                    const int it = b0 + i;
                    if (((taken[l] >> it) & 1u) || bank[l][it] != (uint8_t)best) continue;
                    taken[l] |= 1u << it;
                    outp[l][st] = srcp[l][it];
                    break;
                }
                if (inA) {
                    --ra[l];
                } else {
                    if (split[l] == PC) split[l] = st;
                    --rb[l];
                }
                ++load[best];
            }
        }
        for (int l = 0; l < 32; ++l) {
            uint32_t ow[32], oo[32];
            for (int k = 0; k < PC; ++k) {
                const int pos = c * PC + k;
                ow[k] = im[(size_t)pos * ROW_NT + l];
                const uint32_t o2 = im[(size_t)(64 + pos / 2) * ROW_NT + l];
                oo[k] = (pos & 1) ? (o2 >> 16) : (o2 & 0xffffu);
            }
            for (int k = 0; k < PC; k += 2) {
                uint32_t wk[2], ok[2];
                for (int h = 0; h < 2; ++h) {
                    const uint32_t src = outp[l][k + h];
                    wk[h] = (src & 0x80u) ? 0u : ow[src];
                    ok[h] = (src & 0x80u) ? 4u * (src & 31u) : oo[src];
                }
                const int pos = c * PC + k;
                im[(size_t)pos * ROW_NT + l] = wk[0];
                im[(size_t)(pos + 1) * ROW_NT + l] = wk[1];
                im[(size_t)(64 + pos / 2) * ROW_NT + l] = (ok[0] & 0xffffu) | (ok[1] << 16);
            }
            uint32_t sp = me[4 * l + 1];
            sp = (sp & ~(0xffu << (8 * c))) | ((uint32_t)split[l] << (8 * c));
            me[4 * l + 1] = sp;
        }
        }
    }
}

}  // namespace sdnn
