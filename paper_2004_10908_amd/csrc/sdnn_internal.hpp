// Internal declarations shared by the kernels and the host side of the library.
// Not part of the public ABI (include/sdnn.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdnn {

constexpr int K = 32;                    // inputs per neuron (the only supported k)
constexpr int LDS_BYTES = 160 * 1024;    // gfx950 LDS per workgroup
constexpr int MAX_BATCHES = 256;
constexpr int BAR_WORDS = 10 * 32;       // grid-barrier words (10 lines of 128 B)

// Arguments of one forward layer over a set of rows.
//  Row ids index the [*][N] buffers; row p of the work list is
//    list_in ? list_in[p] : row_base + p,   p < (cnt_in ? *cnt_in : nrows).
struct LayerArgs {
    const float* yin;        // activations entering the layer
    float* yout;             // activations leaving it (same row ids)
    float* ycopy;            // optional second copy of the output rows (checkpoint), or null
    int32_t dead_mark;       // value written to alive[row] for a row found all-zero here: 0, or -1
                             // where the final output buffer still holds the row's older values
                             // (the finalize pass zeroes those rows; no layer writes its own input)
    const int32_t* idx;      // [N][K] this layer
    const float* w;          // [N][K]
    const float* b;          // [N]
    const int32_t* list_in;  // work list (null = identity)
    int32_t* list_out;       // rows with a nonzero output are appended here (null = no compaction)
    const int32_t* cnt_in;   // device row count of the work list (null = nrows)
    int32_t* cnt_out;        // append counter for list_out
    int32_t* alive;          // alive[row] = output row nonzero (or null)
    int32_t row_base;
    int32_t nrows;
    int32_t N;
    int32_t layer;
    float clamp;
    // scheduled (resident-weight) kernel only; ignored by the others
    const uint32_t* ent;         // [SCHED_DSTORE][npad] slot schedule of this layer (step-major: coalesced)
    const int32_t* lane_neuron;  // [npad] neuron of each lane slot (-1: none)
    const int32_t* wave_steps;   // [nblk] steps of each 64-neuron block
    int32_t* tile_bits;          // [max tiles] (parts done << 16) | per-part row bits, zero between layers
    int32_t* prog;               // [streams][4] tile counts of the parts of each tile stream (lockstep hint)
    int32_t parts;               // G: workgroups sharing a tile (each owns NT neurons)
    int32_t nblk;                // 64-neuron blocks
    // linear (input-gradient) use of the scheduled kernel: weights come from
    // w[ent_w[...]] and output row p goes to rows_out[p] (or p)
    const uint32_t* ent_w;
    const int32_t* rows_out;
    // wide-layer kernels only: packed row tiles [tile][N][T] and two words per tile
    // (row bits, workgroups done), zero between layers
    float* packed;
    int32_t* wide_words;
    // one-row-tile kernel only: one word per work-list position (parts done << 16 |
    // parts with a nonzero output), zero between layers
    int32_t* row_words;
    int32_t row_parts;           // G: parts of ROW_PART neurons sharing a row
    const uint8_t* row_perm;     // [N][K] slot order of this layer (bank-scheduled variant), or null
    // chunked one-row-tile kernel only, this layer's lane images built at create time:
    // [parts][ROWC_IMG][ROW_NT] register words (64 weights, 32 packed offsets),
    // [parts][ROW_NT][4] pair words (neurons, split, overflow counts, first entry),
    // [parts][ROWC_OVF_CAP][2] overflow entries
    const uint32_t* rowc_img;
    const uint32_t* rowc_meta;
    const uint32_t* rowc_ovf;
};

// Scheduled weight-gradient pass over one layer (rows are compact 0..R-1).
struct SchedDwArgs {
    const float* y_in;           // [R][N] Y_l
    const float* y_out;          // [R][N] Y_{l+1} (mask)
    const float* dy;             // [R][N] dL/dY_{l+1}
    float* g_out;                // [R][N] masked gradient G (written)
    const int32_t* nrows;        // device R
    const uint32_t* ent;         // forward schedule of the layer
    const int32_t* lane_neuron;
    const int32_t* wave_steps;
    float* pdw;                  // [S][N][K] per-stream partials
    float* pdb;                  // [S][N]
    int32_t N;
    int32_t parts;
    int32_t nblk;
    float clamp;
};

constexpr int SCHED_T = 4;       // rows per tile of the scheduled kernel
constexpr int SCHED_NT = 512;    // its workgroup size (each lane owns two neurons)
constexpr int SCHED_DMAX = 40;   // schedule steps held in registers
constexpr int SCHED_DSTORE = 64; // schedule steps stored per lane
// register steps of the input-gradient kernel's two blocks per wave: the transposed
// schedule puts a wave's 64 highest-degree input neurons in its even block
constexpr int SCHED_DMAX_T0 = 52;
constexpr int SCHED_DMAX_T1 = 36;
constexpr int SCHED_OVF = 30;    // block-steps past SCHED_DMAX a workgroup keeps in LDS (512 bytes each)
constexpr int SCHED_SCALARS = 128; // bytes of per-workgroup scalars after the tile buffers
constexpr int SCHED_PROG = 1024;   // ints of the parts' progress words ([streams][4])
constexpr int SCHED_PART = 1024;   // neurons per workgroup ("part") of the scheduled kernels
constexpr int SCHED_OUT = SCHED_T * SCHED_PART * 4;   // bytes of the output staging tile

// The two tile buffers of the scheduled kernels: 4 rows of N floats each, stored
// [id][row] (16 bytes per id) in blocks of 64 ids, the blocks of the two buffers
// interleaved (block m of buffer b at byte 2048 m + 1024 b).
__host__ __device__ inline size_t sched_tile_bytes(int N) { return (size_t)2048 * (size_t)((N + 63) / 64); }
// LDS byte offset of input id in buffer 0 (buffer 1: + 1024)
__host__ __device__ inline uint32_t sched_slot_offset(uint32_t id) { return ((id >> 6) << 11) | ((id & 63u) << 4); }

// LDS of the scheduled forward kernel: the tile buffers, the scalars, the output
// staging tile, the overflow area.
inline size_t sched_lds_bytes(int N) {
    return sched_tile_bytes(N) + SCHED_SCALARS + SCHED_OUT + (size_t)SCHED_OVF * 512;
}

// Whole forward pass run by the persistent kernel (all layers, one launch).
struct ChainArgs {
    const float* y0;         // [rows][N] input
    float* y_out;            // [rows][N] output, ping-pong buffer "X"
    float* act;              // [rows][N] workspace ping-pong buffer
    float* ckpt;             // checkpoints or null
    const int32_t* idx;      // [L][N][K]
    const float* w;          // [L][N][K]
    const float* b;          // [L][N]
    int32_t* list0;          // [rows]
    int32_t* list1;          // [rows]
    int32_t* cnt;            // [L+1]
    int32_t* alive;          // [rows]
    unsigned* bar;           // barrier words (see grid_barrier)
    int32_t* err;            // device error word
    int32_t rows;
    int32_t N;
    int32_t L;
    int32_t ckpt_every;
    int32_t compaction;
    float clamp;
    // scheduled kernel only (stacked over layers)
    const uint32_t* ent;         // [L][SCHED_DSTORE][npad]
    const int32_t* lane_neuron;  // [L][npad]
    const int32_t* wave_steps;   // [L][nblk]
    int32_t* tile_bits;
    int32_t* prog;
    int32_t parts;
    int32_t nblk;
    // wide-layer kernels only
    float* packed;
    int32_t* wide_words;
    // one-row-tile kernel only
    int32_t* row_words;
    int32_t row_parts;
    const uint8_t* row_perm;     // [L][N][K] slot orders (bank-scheduled variant), or null
    const uint32_t* rowc_img;    // chunked one-row-tile kernel: the lane images of every layer (see LayerArgs)
    const uint32_t* rowc_meta;
    const uint32_t* rowc_ovf;
};

// Error codes written to the device error word.
enum DeviceError : int32_t { DEV_OK = 0, DEV_BARRIER_TIMEOUT = 1 };

// Kernel variant table (instantiated in sdnn_fwd.hip).
struct FwdVariant {
    int T;          // rows per tile
    int NT;         // threads per workgroup
    int staged;     // 7 = as 6, two parts per workgroup, one weight per layer;
                    // 6 = one-row tiles staged in T chunks (rows wider than one LDS buffer),
                    // ascending order; 5 = one-row tiles, bank-scheduled slot order; 4 = one-row tiles
                    // (resident weights), ascending order; 3 = wide (packed row tiles),
                    // 2 = scheduled resident-weight kernel,
                    // 1 = rows staged in LDS, 0 = direct gather
    const void* layer_fn;    // __global__ void(LayerArgs)
    const void* chain_fn;    // __global__ void(ChainArgs)  (cooperative)
    const void* pack_fn;     // wide only: __global__ void(LayerArgs), launched before layer_fn
};
// rows per tile of the wide-layer kernels (the packed buffer and the tile words are
// sized for the smallest and the largest)
constexpr int WIDE_TMIN = 8;
constexpr int WIDE_TMAX = 32;
constexpr int WIDE_PACK_NT = 256;    // threads of the pack kernel
// The one-row-tile resident-weight kernel (sdnn_row.hip): a workgroup of ROW_NT
// lanes owns ROW_PART neurons (two per lane, ids and weights in registers) and
// stages one activation row at a time in LDS; ceil(N / ROW_PART) parts share a row.
constexpr int ROW_NT = 1024;
constexpr int ROW_PART = 2048;
constexpr int ROW_NMAX = 16384;                          // the row (4 N bytes) fits one 64 KB buffer
constexpr uint32_t ROW_BUF_BYTES = 65536;                // two row buffers at 0 and 65536
constexpr uint32_t ROW_STAGE = 2 * ROW_BUF_BYTES;        // two output stages of ROW_PART floats
constexpr uint32_t ROW_SCAL = ROW_STAGE + 2 * ROW_PART * 4;
constexpr size_t ROW_LDS = ROW_SCAL + 256;
constexpr int ROW_GRID = 256;                            // one workgroup per CU, 8 XCDs x 32
// The chunked one-row-tile kernel (sdnn_rowc.hip): the same parts of ROW_PART
// neurons and ROW_NT lanes, for rows of 16384 < N <= 65536 floats staged in C = 2
// or 4 chunks of N / C ids through the two row buffers.  A part's neurons form
// ROW_NT pairs, one per lane; a pair's slots sit in 64 register positions, 64 / C
// per chunk (first neuron's slots of the chunk, then the second's, padding of
// weight 0, each part in a create-time order that spreads a half-wave's LDS reads
// over the banks); slots past a chunk's positions ("overflow") are kept as
// (weight, offset | owner << 16) entries in LDS after the scalars.  The register
// images are built once per net (k_rowc_build, then k_rowc_sched) from the ids,
// the weights and the pairs the host chose.
constexpr int ROWC_NMAX = 65536;
constexpr int ROWC_IMG = 96;                                             // register words per lane
constexpr uint32_t ROWC_OVF = ROW_SCAL + 256;                            // overflow entries (8 bytes)
constexpr int ROWC_OVF_CAP = (int)((LDS_BYTES - ROWC_OVF) / 8);          // entries per workgroup
constexpr size_t ROWC_LDS = LDS_BYTES;
template <int C>
__global__ void k_layer_rowc(LayerArgs a);
template <int C>
__global__ void k_chain_rowc(ChainArgs c);
__global__ void k_rowc_counts(const int32_t* idx, int64_t neurons, int32_t N, int32_t C, uint32_t* counts);
__global__ void k_rowc_build(const int32_t* idx, const float* w, const uint32_t* pairs, int32_t N, int32_t C,
                             int32_t disp, uint32_t* img, uint32_t* meta, uint32_t* ovf, int32_t* status);
// The uniform-weight two-part kernel (sdnn_rowc.hip): the chunked kernel's lane
// images, two parts per workgroup (4096 neurons), for nets whose layers each have a
// single weight value; N % 4096 == 0.
// The last RU_ZERO ids of every chunk are staged outside the buffer (zero words in
// their place, one per LDS bank); a workgroup's two overflow lists take at most
// RU_OVF_CAP 4-byte entries each, beside the side slots at the end of LDS.
constexpr int RU_ZERO = 32;
constexpr int RU_OVF_CAP = (int)((LDS_BYTES - 2 * 4 * RU_ZERO - ROWC_OVF) / 8);
template <int C>
__global__ void k_layer_rowu(LayerArgs a);
template <int C>
__global__ void k_chain_rowu(ChainArgs c);
__global__ void k_rowu_pads(uint32_t* img, int64_t lanes, uint32_t zoff);
__global__ void k_weights_uniform(const float* w, int64_t per_layer, int64_t total, int32_t* flags);
__global__ void k_rowc_sched(uint32_t* img, uint32_t* meta, int64_t tasks, int32_t C);
// neuron pairs of the chunked kernel from per-neuron chunk counts (byte c of
// counts[l][j] = slots of neuron j of layer l in chunk c): pairs [L][N / 2]; returns
// the largest number of overflow entries of any part of any layer
int build_rowc_pairs(const uint32_t* counts, int N, int L, int C, uint32_t* pairs);
__global__ void k_layer_row(LayerArgs a);
__global__ void k_chain_row(ChainArgs c);
__global__ void k_layer_row_sched(LayerArgs a);
__global__ void k_chain_row_sched(ChainArgs c);
// slot orders of the bank-scheduled one-row-tile kernel (sdnn_rowsched.hip):
// perm [L][N][K]; returns the summed cost in LDS passes
int64_t build_row_schedule(const int32_t* idx, int N, int L, uint8_t* perm);

int fwd_variant_count();
const FwdVariant& fwd_variant(int i);
inline size_t fwd_lds_bytes(const FwdVariant& v, int N) {
    if (v.staged == 4 || v.staged == 5) return ROW_LDS;
    if (v.staged == 6 || v.staged == 7) return ROWC_LDS;
    return v.staged == 2 ? sched_lds_bytes(N) : (v.staged == 1 ? (size_t)v.T * N * sizeof(float) : 0);
}

// Host-side slot scheduling (sdnn_sched.hip): see that file.
int build_schedule(const int32_t* idx, int N, int L, int dmax, uint32_t* ent, int32_t* lane_neuron,
                   int32_t* wave_steps);
int build_transposed_schedule(const int32_t* idx, int N, int L, int dmax, uint32_t* ent, int32_t* lane_input,
                              int32_t* wave_steps);

// Small kernels (sdnn_fwd.hip).
__global__ void k_chain_init(int32_t* cnt, int32_t L, int32_t rows, int32_t compaction, unsigned* bar, int32_t nbar);
constexpr int FIN_BLOCKS = 64;   // workgroups of the finalize passes (each a consecutive row range)
__global__ void k_fin_count(const int32_t* alive, int32_t rows, int32_t* part);
__global__ void k_fin_write(const int32_t* alive, int32_t rows, const int32_t* part, int32_t* nz_rows, int32_t* n_nz,
                            const int32_t* cnt, int32_t n_regions, int32_t L, int32_t* layer_rows,
                            const int32_t* err, int32_t* host_err);
__global__ void k_fin_zero(const int32_t* alive, int32_t rows, int32_t N, float* y_out);
__global__ void k_fill_f32(float* p, int64_t n, float v);
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v);
__global__ void k_check_params(const int32_t* idx, const float* w, const float* b, int32_t N, int32_t L,
                               int32_t* bad, float* max_bias);
__global__ void k_max_bias(const float* b, int64_t n, int32_t* flag_pos);
__global__ void k_mse(const float* y, const float* t, int64_t n, float* dy, float* partial, float scale);
__global__ void k_mse_final(const float* partial, int32_t nparts, float* loss, float inv_n);

// Backward kernels (sdnn_bwd.hip).
struct BwdDwArgs {
    const float* y_in;       // [R][N] compact Y_l
    const float* y_out;      // [R][N] compact Y_{l+1} (mask)
    const float* dy;         // [R][N] compact dL/dY_{l+1}
    const int32_t* idx;      // [N][K]
    const int32_t* nrows;    // device R
    float* pdw;              // [P][N][K] partials
    float* pdb;              // [P][N]
    int32_t N;
    int32_t P;               // row groups
    float clamp;
};
struct BwdDyArgs {
    const float* y_out;      // [R][N] Y_{l+1}
    const float* dy;         // [R][N] dL/dY_{l+1}
    const int32_t* tr_ptr;   // [N+1]
    const int32_t* tr_e;     // [N*K] edge positions j*K+k grouped by input neuron
    const float* w;          // [N][K]
    const int32_t* nrows;    // device R
    const int32_t* rows_out; // optional: output row r goes to rows_out[r] (scatter), else r
    float* dy_in;            // output dL/dY_l
    int32_t N;
    float clamp;
};
int bwd_T();
int bwd_threads();
const void* bwd_dw_sched_fn();
const void* bwd_dy_sched_fn();
const void* bwd_dw_fn();
const void* bwd_dy_fn();
// sum the first P per-stream partials (with nrows: the first min(P, ceil(*nrows / T)))
__global__ void k_reduce_partials(const float* pdw, const float* pdb, int32_t P, int32_t N, float* dw, float* db,
                                  const int32_t* nrows, int32_t T);
__global__ void k_gather_rows(const float* src, const int32_t* rows, const int32_t* n, int32_t N, float* dst);
__global__ void k_tr_count(const int32_t* idx, int64_t nnz, int32_t* deg);
__global__ void k_tr_scan(const int32_t* deg, int32_t N, int32_t* ptr);
__global__ void k_tr_fill(const int32_t* idx, int64_t nnz, const int32_t* ptr, int32_t* cursor, int32_t* tr_e);
__global__ void k_tr_sort(const int32_t* ptr, int32_t N, int32_t* tr_e);

}  // namespace sdnn
