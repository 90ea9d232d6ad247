// Host side of the C ABI declared in include/sdnn.h: validation, workspace
// layout, the three ways of running the layer chain (eager launches, one
// explicitly built hipGraph, one persistent cooperative kernel), the backward
// orchestration with checkpoint segments, and the tile autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "sdnn.h"
#include "sdnn_internal.hpp"

using namespace sdnn;

namespace {

thread_local std::string g_err;

sdnn_status fail(sdnn_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail(SDNN_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

#define TRY(expr)                                  \
    do {                                           \
        sdnn_status s_ = (expr);                   \
        if (s_ != SDNN_OK) return s_;              \
    } while (0)

constexpr size_t ALIGN = 256;
constexpr int P_GROUPS = 64;                    // backward row groups (dW partials)
constexpr int NBAR = BAR_WORDS;
constexpr size_t LDS_BUDGET = 160 * 1024;       // dynamic LDS a workgroup may use (gfx950 maximum)
constexpr int MSE_BLOCKS = 256;
constexpr int SCHED_GRID = 256;                 // workgroups of the scheduled kernels (8 XCDs x 32)
constexpr int WIDE_DEFAULT_T = 32;               // default tile of the wide-layer kernels (before tuning)
constexpr int WIDE_DEFAULT_NT = 1024;

size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

struct Layout {
    size_t act = 0, list0 = 0, list1 = 0, alive = 0, cnt = 0, bar = 0, err = 0, flag = 0, fin = 0;
    size_t ent = 0, lane_neuron = 0, wave_steps = 0, tile_bits = 0, prog = 0;
    size_t ent_t = 0, ent_w = 0, lane_input = 0, steps_t = 0, gbuf2 = 0;
    bool sched = false;
    bool wide = false;
    size_t packed = 0, wide_words = 0;
    bool row = false, row_sched = false, rowc = false;
    size_t row_words = 0, row_perm = 0, rowc_img = 0, rowc_meta = 0, rowc_ovf = 0;
    size_t tr_ptr = 0, tr_e = 0, seg = 0, gbuf0 = 0, gbuf1 = 0, pdw = 0, pdb = 0;
    size_t total = 0;
};

bool trainable(const sdnn_desc& d) { return (d.flags & SDNN_TRAINABLE) != 0; }

// The scheduled resident-weight kernel needs two 4-row tiles in LDS, ids in
// groups of 16, and at most 4 parts of 1024 neurons (grid of 256 = 8 XCDs x 32).
int sched_parts(const sdnn_desc& d) { return ((d.n_neurons + 63) / 64 + 15) / 16; }

// [L][npad][SCHED_DSTORE] (as the scheduler writes it) -> [L][SCHED_DSTORE][npad]
void step_major(std::vector<uint32_t>& e, int L, size_t npad) {
    std::vector<uint32_t> t(e.size());
    for (int l = 0; l < L; ++l)
        for (size_t sl = 0; sl < npad; ++sl)
            for (int st = 0; st < SCHED_DSTORE; ++st)
                t[((size_t)l * SCHED_DSTORE + st) * npad + sl] = e[((size_t)l * npad + sl) * SCHED_DSTORE + st];
    e.swap(t);
}

bool sched_shape(const sdnn_desc& d) {
    const int nblk = (d.n_neurons + 63) / 64;
    const int G = (nblk + 15) / 16;
    // the tile copies address a row as a 32-bit byte offset from the activation base
    const bool offs32 = (int64_t)std::max<int64_t>(d.max_rows, 1) * d.n_neurons * 4 <= ((int64_t)1 << 32);
    return d.n_neurons % 16 == 0 && sched_lds_bytes(d.n_neurons) <= LDS_BUDGET && (G == 1 || G == 2 || G == 4) &&
           offs32;
}
bool sched_possible(const sdnn_desc& d) { return !(d.flags & SDNN_NO_SCHEDULE) && sched_shape(d); }

// The wide-layer kernels (packed row tiles) serve forward-only nets whose shape the
// scheduled kernel cannot take; their packed buffer holds every row once more.
bool wide_possible(const sdnn_desc& d) { return !trainable(d) && !sched_shape(d); }

// The one-row-tile kernel: a row of N floats fits one 64 KB LDS buffer (so every
// 4-byte offset fits 16 bits), whole 16-byte copies (N % 4 == 0), and at least two
// parts (below that the scheduled kernels serve the net).
bool row_possible(const sdnn_desc& d) {
    return !trainable(d) && d.n_neurons % 4 == 0 && d.n_neurons > ROW_PART && d.n_neurons <= ROW_NMAX;
}
int row_parts(const sdnn_desc& d) { return (d.n_neurons + ROW_PART - 1) / ROW_PART; }

// The chunked one-row-tile kernel: rows wider than one LDS buffer, staged in 2 or 4
// chunks of at most 16384 ids; whole parts (N % 2048 == 0); a create-time pairing
// of the neurons (so not with SDNN_NO_SCHEDULE, whose ids may change).
bool rowc_possible(const sdnn_desc& d) {
    return !trainable(d) && !(d.flags & SDNN_NO_SCHEDULE) && d.n_neurons % ROW_PART == 0 &&
           d.n_neurons > ROW_NMAX && d.n_neurons <= ROWC_NMAX;
}
int rowc_chunks(const sdnn_desc& d) { return d.n_neurons <= 2 * ROW_NMAX ? 2 : 4; }

Layout make_layout(const sdnn_desc& d) {
    Layout y;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return o;
    };
    const size_t R = (size_t)std::max<int64_t>(d.max_rows, 1), N = d.n_neurons, L = d.n_layers;
    y.act = take(R * N * 4);
    y.list0 = take(R * 4);
    y.list1 = take(R * 4);
    y.alive = take(R * 4);
    y.cnt = take((size_t)MAX_BATCHES * (L + 1) * 4);
    y.sched = sched_possible(d);
    if (y.sched) {
        const size_t nblk = (N + 63) / 64, npad = nblk * 64;
        y.ent = take(L * npad * SCHED_DSTORE * 4);
        y.lane_neuron = take(L * npad * 4);
        y.wave_steps = take(L * nblk * 4);
        y.tile_bits = take(((R + SCHED_T - 1) / SCHED_T) * 4);
        y.prog = take(SCHED_PROG * 4);
    }
    y.wide = wide_possible(d);
    if (y.wide) {
        const size_t rt = (R + WIDE_TMAX - 1) / WIDE_TMAX * WIDE_TMAX;
        y.packed = take(rt * N * 4);
        y.wide_words = take(2 * ((R + WIDE_TMIN - 1) / WIDE_TMIN) * 4);
    }
    y.row = row_possible(d);
    y.rowc = rowc_possible(d);
    if (y.row || y.rowc) y.row_words = take(R * 4);
    // the chunked kernel's lane images of every layer (register words, pair words,
    // overflow lists): 400 bytes per pair of neurons and 16 KB per part
    if (y.rowc) {
        const size_t parts = N / ROW_PART;
        y.rowc_img = take(L * parts * ROWC_IMG * ROW_NT * 4);
        y.rowc_meta = take(L * parts * ROW_NT * 16);
        y.rowc_ovf = take(L * parts * ROWC_OVF_CAP * 8);
    }
    // the bank-scheduled slot order of every layer (32 bytes per neuron)
    y.row_sched = y.row && !(d.flags & SDNN_NO_SCHEDULE);
    if (y.row_sched) y.row_perm = take(L * N * K);
    y.bar = take(NBAR * 4);
    y.fin = take(FIN_BLOCKS * 4);
    y.err = take(64);
    y.flag = take(64);
    if (trainable(d)) {
        y.tr_ptr = take(L * (N + 1) * 4);
        y.tr_e = take(L * N * K * 4);
        y.seg = take((size_t)(d.ckpt_every + 1) * R * N * 4);
        y.gbuf0 = take(std::max<size_t>(R, 2) * N * 4);   // also create-time scratch for 2N ints
        y.gbuf1 = take(R * N * 4);
        // dW/db partials: 64 row groups, or one per tile stream of the scheduled kernel
        const size_t groups = std::max<size_t>(P_GROUPS, y.sched ? (size_t)SCHED_GRID / sched_parts(d) : 0);
        y.pdw = take(groups * N * K * 4);
        y.pdb = take(groups * N * 4);
        if (y.sched) {
            const size_t nblk = (N + 63) / 64, npad = nblk * 64;
            y.ent_t = take(L * npad * SCHED_DSTORE * 4);
            y.ent_w = take(L * npad * SCHED_DSTORE * 4);
            y.lane_input = take(L * npad * 4);
            y.steps_t = take(L * nblk * 4);
            y.gbuf2 = take(R * N * 4);
        }
    }
    y.total = off;
    return y;
}

sdnn_status check_desc(const sdnn_desc* d) {
    if (!d) return fail(SDNN_EINVAL, "desc is NULL");
    if (d->k != K) return fail(SDNN_EUNSUPPORTED, "k = %d: only k = 32 inputs per neuron is supported", d->k);
    if (d->n_neurons < 1 || d->n_neurons > (1 << 20)) return fail(SDNN_EINVAL, "n_neurons = %d out of [1, 2^20]", d->n_neurons);
    if (d->n_layers < 1) return fail(SDNN_EINVAL, "n_layers = %d must be >= 1", d->n_layers);
    if (d->n_neurons < K) return fail(SDNN_EINVAL, "n_neurons = %d < k: k distinct inputs impossible", d->n_neurons);
    if (!(d->clamp > 0.f) || !std::isfinite(d->clamp)) return fail(SDNN_EINVAL, "clamp must be finite and > 0");
    if (d->max_rows < 0 || d->max_rows > INT32_MAX) return fail(SDNN_EINVAL, "max_rows out of range");
    if ((double)d->max_rows * d->n_neurons >= 9.0e15) return fail(SDNN_EINVAL, "max_rows * n_neurons too large");
    if (trainable(*d)) {
        if (d->ckpt_every < 1) return fail(SDNN_EINVAL, "SDNN_TRAINABLE needs ckpt_every >= 1");
        if ((size_t)bwd_T() * d->n_neurons * 4 > LDS_BUDGET)
            return fail(SDNN_EUNSUPPORTED, "backward supports n_neurons <= %zu", LDS_BUDGET / (bwd_T() * 4));
    } else if (d->ckpt_every < 0) {
        return fail(SDNN_EINVAL, "ckpt_every must be >= 0");
    }
    if (d->flags & ~(SDNN_TRAINABLE | SDNN_NO_COMPACTION | SDNN_DEBUG_CHECKS | SDNN_AUTOTUNE | SDNN_NO_SCHEDULE))
        return fail(SDNN_EINVAL, "unknown flag bits 0x%x", d->flags);
    return SDNN_OK;
}

// ---------------------------------------------------------------- launch records
// A kernel launch with its arguments kept alive, so it can be issued eagerly or
// recorded as a hipGraph kernel node.
struct Launch {
    virtual ~Launch() = default;
    const void* fn = nullptr;
    dim3 grid, block;
    size_t shmem = 0;
    bool cooperative = false;
    bool timed = false;                 // bracketed by timing events when the net's timing is on
    std::vector<void*> ptrs;
};

template <typename... A>
struct LaunchT : Launch {
    std::tuple<A...> args;
    explicit LaunchT(A... a) : args(a...) {
        std::apply([this](auto&... x) { ptrs = {static_cast<void*>(&x)...}; }, args);
    }
};

template <typename... A>
std::unique_ptr<Launch> mk(const void* fn, dim3 grid, dim3 block, size_t shmem, A... a) {
    auto p = std::make_unique<LaunchT<A...>>(a...);
    p->fn = fn;
    p->grid = grid;
    p->block = block;
    p->shmem = shmem;
    return p;
}

using Plan = std::vector<std::unique_ptr<Launch>>;

}  // namespace

struct sdnn_net_s {
    sdnn_desc d{};
    const int32_t* idx = nullptr;
    const float* w = nullptr;
    const float* b = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    Layout lay;
    float* act = nullptr;
    int32_t *list0 = nullptr, *list1 = nullptr, *alive = nullptr, *cnt = nullptr, *err = nullptr, *flag = nullptr;
    int32_t* fin = nullptr;             // per-range alive counts of the finalize passes
    int32_t* herr = nullptr;            // pinned host word: the device error as the finalize pass published it
    int32_t* herr_dev = nullptr;        // its device address
    unsigned* bar = nullptr;
    int32_t *tr_ptr = nullptr, *tr_e = nullptr;
    float *seg = nullptr, *gbuf0 = nullptr, *gbuf1 = nullptr, *pdw = nullptr, *pdb = nullptr;
    bool compaction = true;
    bool sched = false;                 // scheduled kernel available (schedule built)
    bool wide = false;                  // wide-layer kernels available (packed buffer present)
    float* packed = nullptr;
    int32_t* wide_words = nullptr;
    bool row = false;                   // one-row-tile kernel available
    int32_t* row_words = nullptr;
    int row_parts = 0;
    uint8_t* row_perm = nullptr;        // its bank-scheduled slot orders (null: ascending only)
    bool rowc = false;                  // chunked one-row-tile kernel available (images built)
    uint32_t *rowc_img = nullptr, *rowc_meta = nullptr, *rowc_ovf = nullptr;   // its lane images [L][...]
    int rowc_chunks = 0;
    bool rowu = false;                  // every layer has one weight value: the two-part kernel serves it
    uint32_t* ent = nullptr;
    int32_t *lane_neuron = nullptr, *wave_steps = nullptr, *tile_bits = nullptr, *prog = nullptr;
    int parts = 1, nblk = 0;
    bool sched_bwd = false;             // transposed schedule built (scheduled backward)
    uint32_t *ent_t = nullptr, *ent_w = nullptr;
    int32_t *lane_input = nullptr, *steps_t = nullptr;
    float* gbuf2 = nullptr;
    int exec = SDNN_EXEC_AUTO;
    int variant = 0;
    int grid = 0;
    int chain_grid = 0;
    float tuned_us = 0.f;
    int num_cu = 0;
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<int64_t> gkey;
    bool timing = false;                 // sdnn_set_timing
    std::vector<hipEvent_t> tev;         // start/stop pairs, created on first use
    size_t tev_used = 0;                 // events recorded since the last sdnn_kernel_time
    ~sdnn_net_s() {
        if (herr) (void)hipHostFree(herr);
    }
};

namespace {

const FwdVariant& var(const sdnn_net_s* n) { return fwd_variant(n->variant); }

// SDNN_EDEVICE if a kernel of an earlier call raised the device error word and the
// finalize pass of a forward (or sdnn_check_device) has published it to the host.
sdnn_status host_error(const sdnn_net_s* n) {
    const int32_t e = n->herr ? __atomic_load_n(n->herr, __ATOMIC_ACQUIRE) : 0;
    if (e == DEV_BARRIER_TIMEOUT) return fail(SDNN_EDEVICE, "a persistent-kernel grid barrier timed out in an earlier call");
    if (e != 0) return fail(SDNN_EDEVICE, "device error %d raised in an earlier call", e);
    return SDNN_OK;
}

bool variant_fits(const sdnn_net_s* n, const FwdVariant& v) {
    if (v.staged == 7) return n->rowc && n->rowu && v.T == n->rowc_chunks;
    if (v.staged == 6) return n->rowc && v.T == n->rowc_chunks;
    if (v.staged == 5) return n->row && n->row_perm;
    if (v.staged == 4) return n->row;
    if (v.staged == 3) return n->wide;
    if (v.staged == 2) return n->sched;
    if (!v.staged) return true;
    return (size_t)v.T * n->d.n_neurons * 4 <= LDS_BUDGET;
}

// Schedule fields of layer l (the scheduled kernel reads them; others ignore them).
void fill_sched(const sdnn_net_s* n, LayerArgs& a, int l) {
    a.packed = n->packed;
    a.wide_words = n->wide_words;
    a.row_words = n->row_words;
    a.row_parts = n->row_parts;
    a.row_perm = n->row_perm ? n->row_perm + (size_t)l * n->d.n_neurons * K : nullptr;
    if (n->rowc) {
        const size_t parts = (size_t)n->row_parts;
        a.rowc_img = n->rowc_img + (size_t)l * parts * ROWC_IMG * ROW_NT;
        a.rowc_meta = n->rowc_meta + (size_t)l * parts * ROW_NT * 4;
        a.rowc_ovf = n->rowc_ovf + (size_t)l * parts * ROWC_OVF_CAP * 2;
    }
    if (!n->sched) return;
    const size_t npad = (size_t)n->nblk * 64;
    a.ent = n->ent + (size_t)l * npad * SCHED_DSTORE;
    a.lane_neuron = n->lane_neuron + (size_t)l * npad;
    a.wave_steps = n->wave_steps + (size_t)l * n->nblk;
    a.tile_bits = n->tile_bits;
    a.prog = n->prog;
    a.parts = n->parts;
    a.nblk = n->nblk;
}

// Workgroups of a layer launch: grid-stride kernels shrink to the tile count; the
// scheduled kernel keeps its full (XCD x part) grid and idle workgroups exit.
int launch_grid(const sdnn_net_s* n, const FwdVariant& v, int64_t rows) {
    if (v.staged >= 2) return n->grid;
    return (int)std::max<int64_t>(1, std::min<int64_t>(n->grid, (rows + v.T - 1) / v.T));
}

sdnn_status prepare_variant(sdnn_net_s* n, int vi, int* grid, int* chain_grid) {
    const FwdVariant& v = fwd_variant(vi);
    const size_t sh = fwd_lds_bytes(v, n->d.n_neurons);
    HIPCHK(hipFuncSetAttribute(v.layer_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
    HIPCHK(hipFuncSetAttribute(v.chain_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
    int occ = 0, occc = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, v.layer_fn, v.NT, sh));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occc, v.chain_fn, v.NT, sh));
    if (occ < 1 || occc < 1) return fail(SDNN_EUNSUPPORTED, "kernel variant T=%d NT=%d does not fit a CU", v.T, v.NT);
    *grid = n->num_cu * occ;
    *chain_grid = n->num_cu * occc;
    if (v.staged == 2) {
        // the scheduled kernels map workgroups to (XCD, part, stream): 8 * parts must divide the grid
        if (*grid < SCHED_GRID || *chain_grid < SCHED_GRID)
            return fail(SDNN_EUNSUPPORTED, "scheduled kernel needs %d co-resident workgroups", SCHED_GRID);
        *grid = SCHED_GRID;
        *chain_grid = SCHED_GRID;
    }
    if (v.staged >= 4 && v.staged <= 7) {
        // one workgroup per CU, mapped to (XCD, part, stream) like the scheduled kernels
        if (*grid < ROW_GRID || *chain_grid < ROW_GRID)
            return fail(SDNN_EUNSUPPORTED, "one-row-tile kernel needs %d co-resident workgroups", ROW_GRID);
        *grid = ROW_GRID;
        *chain_grid = ROW_GRID;
    }
    return SDNN_OK;
}

// Default tile plan: the scheduled kernel when its schedule exists, else the
// widest power-of-two row tile that fits the LDS budget.
int default_variant(const sdnn_net_s* n) {
    const int N = n->d.n_neurons;
    if (n->sched)
        for (int i = 0; i < fwd_variant_count(); ++i)
            if (fwd_variant(i).staged == 2) return i;
    if (n->row)
        for (int want : {5, 4}) {
            if (want == 5 && !n->row_perm) continue;
            for (int i = 0; i < fwd_variant_count(); ++i)
                if (fwd_variant(i).staged == want) return i;
        }
    // the two-part kernel stages each row half as often (C4 layer: 6.6 against 10.3 ms)
    if (n->rowc)
        for (int want : {7, 6}) {
            if (want == 7 && !n->rowu) continue;
            for (int i = 0; i < fwd_variant_count(); ++i)
                if (fwd_variant(i).staged == want && fwd_variant(i).T == n->rowc_chunks) return i;
        }
    int best = -1, bestT = 0;
    for (int i = 0; i < fwd_variant_count(); ++i) {
        const FwdVariant& v = fwd_variant(i);
        if (v.staged != 1 || (size_t)v.T * N * 4 > LDS_BUDGET || v.T > 16) continue;
        const int want_nt = v.T >= 16 ? 512 : 1024;
        if (v.NT != want_nt) continue;
        if (v.T > bestT) { bestT = v.T; best = i; }
    }
    // where not even 2 rows fit LDS the packed tiles win by far (65536 neurons: 16.0
    // ms per 15000-row layer against 315 ms for 4-byte gathers straight from the
    // rows).  At 16384 neurons they are ahead on a full-live layer (13.6 against 15.6
    // ms per 60000-row layer) but behind on the whole forward, where every empty
    // layer costs them two launches (pack and compute) instead of one
    if (n->wide && bestT < 2)
        for (int i = 0; i < fwd_variant_count(); ++i) {
            const FwdVariant& v = fwd_variant(i);
            if (v.staged == 3 && v.T == WIDE_DEFAULT_T && v.NT == WIDE_DEFAULT_NT) return i;
        }
    if (best >= 0) return best;
    for (int i = 0; i < fwd_variant_count(); ++i) {
        const FwdVariant& v = fwd_variant(i);
        if (!v.staged && v.T == 1 && v.NT == 1024) return i;
    }
    return 0;
}

// Workgroups of the wide kernels' pack pass over up to `rows` rows.
int pack_grid(const sdnn_net_s* n, const FwdVariant& v, int64_t rows) {
    const int64_t tasks = (rows + v.T - 1) / v.T * ((n->d.n_neurons + 4 * WIDE_PACK_NT - 1) / (4 * WIDE_PACK_NT));
    return (int)std::max<int64_t>(1, std::min<int64_t>(tasks, (int64_t)n->num_cu * 8));
}

// One layer launch of variant v (the wide variants: the pack pass, then the layer).
hipError_t launch_layer(const sdnn_net_s* n, const FwdVariant& v, int grid, LayerArgs& a, int64_t rows, hipStream_t s) {
    void* args[] = {&a};
    if (v.pack_fn) {
        const hipError_t e = hipLaunchKernel(v.pack_fn, dim3(pack_grid(n, v, rows)), dim3(WIDE_PACK_NT), args, 0, s);
        if (e != hipSuccess) return e;
    }
    return hipLaunchKernel(v.layer_fn, dim3(grid), dim3(v.NT), args, fwd_lds_bytes(v, n->d.n_neurons), s);
}

sdnn_status issue(const Plan& plan, hipStream_t s, sdnn_net_s* n = nullptr) {
    for (const auto& L : plan) {
        const bool timed = n && n->timing && L->timed;
        if (timed) {
            if (n->tev_used + 2 > n->tev.size()) {
                for (int i = 0; i < 2; ++i) {
                    hipEvent_t e;
                    HIPCHK(hipEventCreate(&e));
                    n->tev.push_back(e);
                }
            }
            HIPCHK(hipEventRecord(n->tev[n->tev_used], s));
        }
        if (L->cooperative) {
            HIPCHK(hipLaunchCooperativeKernel(L->fn, L->grid, L->block, const_cast<void**>(L->ptrs.data()),
                                              (unsigned)L->shmem, s));
        } else {
            HIPCHK(hipLaunchKernel(L->fn, L->grid, L->block, const_cast<void**>(L->ptrs.data()), L->shmem, s));
        }
        if (timed) {
            HIPCHK(hipEventRecord(n->tev[n->tev_used + 1], s));
            n->tev_used += 2;
        }
    }
    return SDNN_OK;
}

void drop_graph(sdnn_net_s* n) {
    if (n->gexec) (void)hipGraphExecDestroy(n->gexec);
    if (n->graph) (void)hipGraphDestroy(n->graph);
    n->gexec = nullptr;
    n->graph = nullptr;
    n->gkey.clear();
}

sdnn_status build_graph(sdnn_net_s* n, const Plan& plan) {
    drop_graph(n);
    HIPCHK(hipGraphCreate(&n->graph, 0));
    hipGraphNode_t prev = nullptr;
    for (const auto& L : plan) {
        hipKernelNodeParams p{};
        p.func = const_cast<void*>(L->fn);
        p.gridDim = L->grid;
        p.blockDim = L->block;
        p.sharedMemBytes = (unsigned)L->shmem;
        p.kernelParams = const_cast<void**>(L->ptrs.data());
        p.extra = nullptr;
        hipGraphNode_t node;
        HIPCHK(hipGraphAddKernelNode(&node, n->graph, prev ? &prev : nullptr, prev ? 1 : 0, &p));
        prev = node;
    }
    HIPCHK(hipGraphInstantiate(&n->gexec, n->graph, nullptr, nullptr, 0));
    return SDNN_OK;
}

LayerArgs layer_args_chain(const sdnn_net_s* n, int l, const float* y0, float* y_out, float* ckpt, int64_t rows,
                           int32_t row_base, int32_t nb_rows, int32_t* cnt_region) {
    const int L = n->d.n_layers, N = n->d.n_neurons, S = n->d.ckpt_every;
    const size_t NK = (size_t)N * K;
    const bool out_is_y = ((L - 1 - l) & 1) == 0;
    const bool cmp = n->compaction;
    LayerArgs a{};
    a.yin = l == 0 ? y0 : (out_is_y ? n->act : y_out);
    a.yout = out_is_y ? y_out : n->act;
    a.ycopy = (ckpt && S > 0 && (l + 1) % S == 0 && l + 1 < L) ? ckpt + (size_t)((l + 1) / S - 1) * rows * N : nullptr;
    a.dead_mark = (cmp && !out_is_y) ? -1 : 0;
    a.idx = n->idx + l * NK;
    a.w = n->w + l * NK;
    a.b = n->b + (size_t)l * N;
    a.list_in = (l == 0 || !cmp) ? nullptr : ((l & 1) ? n->list1 : n->list0);
    a.list_out = cmp ? (((l + 1) & 1) ? n->list1 : n->list0) : nullptr;
    a.cnt_in = (l == 0 || !cmp) ? nullptr : cnt_region + l;
    a.cnt_out = cnt_region + l + 1;
    a.alive = n->alive;
    a.row_base = row_base;
    a.nrows = nb_rows;
    a.N = N;
    a.layer = l;
    a.clamp = n->d.clamp;
    fill_sched(n, a, l);
    return a;
}

// The finalize passes: alive rows per row range, then the ascending nonzero-row
// ids and the per-layer row profile (summed over `regions` count regions), then the
// clearing of rows that died while the output buffer held their older values.
void push_finalize(Plan& p, const sdnn_net_s* n, int64_t rows, float* y_out, int32_t* nz_rows, int32_t* n_nz,
                   int regions, int32_t* layer_rows) {
    p.push_back(mk((const void*)&k_fin_count, dim3(FIN_BLOCKS), dim3(1024), 0, (const int32_t*)n->alive, (int32_t)rows,
                   n->fin));
    p.push_back(mk((const void*)&k_fin_write, dim3(FIN_BLOCKS), dim3(1024), 0, (const int32_t*)n->alive, (int32_t)rows,
                   (const int32_t*)n->fin, nz_rows, n_nz, (const int32_t*)n->cnt, (int32_t)regions,
                   (int32_t)n->d.n_layers, layer_rows, (const int32_t*)n->err, n->herr_dev));
    if (n->compaction && rows > 0)
        p.push_back(mk((const void*)&k_fin_zero, dim3((unsigned)std::min<int64_t>(rows, 2048)), dim3(256), 0,
                       (const int32_t*)n->alive, (int32_t)rows, (int32_t)n->d.n_neurons, y_out));
}

// The per-batch ("plain") chain: for each non-empty batch, an init node and L
// layer nodes; then one finalize node.  Used eagerly or as one hipGraph.
Plan plan_chain(const sdnn_net_s* n, const float* y0, int64_t rows, const int64_t* off, int nb, float* y_out,
                int32_t* nz_rows, int32_t* n_nz, float* ckpt, int32_t* layer_rows) {
    Plan p;
    const int L = n->d.n_layers;
    const FwdVariant& v = var(n);
    const size_t sh = fwd_lds_bytes(v, n->d.n_neurons);
    int region = 0;
    for (int bi = 0; bi < nb; ++bi) {
        const int32_t r0 = (int32_t)off[bi], nbr = (int32_t)(off[bi + 1] - off[bi]);
        if (nbr == 0) continue;
        int32_t* cr = n->cnt + (size_t)region * (L + 1);
        p.push_back(mk((const void*)&k_chain_init, dim3(1), dim3(256), 0, cr, (int32_t)L, nbr,
                       (int32_t)(n->compaction ? 1 : 0), (unsigned*)nullptr, (int32_t)0));
        for (int l = 0; l < L; ++l) {
            LayerArgs a = layer_args_chain(n, l, y0, y_out, ckpt, rows, r0, nbr, cr);
            if (v.pack_fn) p.push_back(mk(v.pack_fn, dim3(pack_grid(n, v, nbr)), dim3(WIDE_PACK_NT), 0, a));
            p.push_back(mk(v.layer_fn, dim3(launch_grid(n, v, nbr)), dim3(v.NT), sh, a));
        }
        ++region;
    }
    push_finalize(p, n, rows, y_out, nz_rows, n_nz, region, layer_rows);
    return p;
}

// The merged chain: all batches' rows in one work list, one node per layer.
Plan plan_merged(const sdnn_net_s* n, const float* y0, int64_t rows, float* y_out, int32_t* nz_rows, int32_t* n_nz,
                 float* ckpt, int32_t* layer_rows) {
    const int64_t off[2] = {0, rows};
    return plan_chain(n, y0, rows, off, 1, y_out, nz_rows, n_nz, ckpt, layer_rows);
}

Plan plan_persistent(const sdnn_net_s* n, const float* y0, int64_t rows, float* y_out, int32_t* nz_rows,
                     int32_t* n_nz, float* ckpt, int32_t* layer_rows) {
    Plan p;
    const int L = n->d.n_layers;
    const FwdVariant& v = var(n);
    const size_t sh = fwd_lds_bytes(v, n->d.n_neurons);
    p.push_back(mk((const void*)&k_chain_init, dim3(1), dim3(256), 0, n->cnt, (int32_t)L, (int32_t)rows,
                   (int32_t)(n->compaction ? 1 : 0), n->bar, (int32_t)NBAR));
    ChainArgs c{};
    c.y0 = y0;
    c.y_out = y_out;
    c.act = n->act;
    c.ckpt = ckpt;
    c.idx = n->idx;
    c.w = n->w;
    c.b = n->b;
    c.list0 = n->list0;
    c.list1 = n->list1;
    c.cnt = n->cnt;
    c.alive = n->alive;
    c.bar = n->bar;
    c.err = n->err;
    c.rows = (int32_t)rows;
    c.N = n->d.n_neurons;
    c.L = L;
    c.ckpt_every = n->d.ckpt_every > 0 ? n->d.ckpt_every : L + 1;
    c.compaction = n->compaction ? 1 : 0;
    c.clamp = n->d.clamp;
    if (n->sched) {
        c.ent = n->ent;
        c.lane_neuron = n->lane_neuron;
        c.wave_steps = n->wave_steps;
        c.tile_bits = n->tile_bits;
        c.prog = n->prog;
        c.parts = n->parts;
        c.nblk = n->nblk;
    }
    c.packed = n->packed;
    c.wide_words = n->wide_words;
    c.row_words = n->row_words;
    c.row_parts = n->row_parts;
    c.row_perm = n->row_perm;
    c.rowc_img = n->rowc_img;
    c.rowc_meta = n->rowc_meta;
    c.rowc_ovf = n->rowc_ovf;
    auto ch = mk(v.chain_fn, dim3(n->chain_grid), dim3(v.NT), sh, c);
    ch->cooperative = true;
    ch->timed = true;
    p.push_back(std::move(ch));
    push_finalize(p, n, rows, y_out, nz_rows, n_nz, 1, layer_rows);
    return p;
}

int blocks_for(int64_t n, int per = 256, int cap = 4096) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (n + per - 1) / per));
}

// One layer of the scheduled backward: dW/db partials per tile stream (and the
// masked gradient G), their fixed-order reduction, then the input gradient
// through the transposed schedule (scattered to rows_out rows when given).
sdnn_status backward_layer_sched(const sdnn_net_s* n, int l, const float* y_in, const float* y_out, const float* dy,
                                 float* dy_in, const int32_t* rows_out, const int32_t* nrows, int64_t rows, float* dw_l,
                                 float* db_l, hipStream_t s) {
    const int N = n->d.n_neurons;
    const size_t npad = (size_t)n->nblk * 64;
    const size_t sh = sched_lds_bytes(N);
    const int S = SCHED_GRID / n->parts;
    SchedDwArgs da{};
    da.y_in = y_in;
    da.y_out = y_out;
    da.dy = dy;
    da.g_out = n->gbuf2;
    da.nrows = nrows;
    da.ent = n->ent + (size_t)l * npad * SCHED_DSTORE;
    da.lane_neuron = n->lane_neuron + (size_t)l * npad;
    da.wave_steps = n->wave_steps + (size_t)l * n->nblk;
    da.pdw = n->pdw;
    da.pdb = n->pdb;
    da.N = N;
    da.parts = n->parts;
    da.nblk = n->nblk;
    da.clamp = n->d.clamp;
    void* dargs[] = {&da};
    HIPCHK(hipLaunchKernel(bwd_dw_sched_fn(), dim3(SCHED_GRID), dim3(2 * SCHED_NT), dargs, sh, s));
    hipLaunchKernelGGL(k_reduce_partials, dim3(blocks_for((int64_t)N * K + N)), dim3(256), 0, s, (const float*)n->pdw,
                       (const float*)n->pdb, (int32_t)S, (int32_t)N, dw_l, db_l, nrows, (int32_t)SCHED_T);
    if (dy_in) {
        LayerArgs a{};
        a.yin = n->gbuf2;
        a.yout = dy_in;
        a.w = n->w + (size_t)l * N * K;
        a.cnt_in = nrows;
        a.N = N;
        a.layer = l;
        a.clamp = n->d.clamp;
        a.ent = n->ent_t + (size_t)l * npad * SCHED_DSTORE;
        a.ent_w = n->ent_w + (size_t)l * npad * SCHED_DSTORE;
        a.lane_neuron = n->lane_input + (size_t)l * npad;
        a.wave_steps = n->steps_t + (size_t)l * n->nblk;
        a.parts = n->parts;
        a.nblk = n->nblk;
        a.rows_out = rows_out;
        void* yargs[] = {&a};
        HIPCHK(hipLaunchKernel(bwd_dy_sched_fn(), dim3(SCHED_GRID), dim3(SCHED_NT), yargs, sched_lds_bytes(N), s));
    }
    (void)rows;
    HIPCHK(hipGetLastError());
    return SDNN_OK;
}

}  // namespace

// ============================================================================ C ABI
extern "C" {

const char* sdnn_last_error(void) { return g_err.c_str(); }

const char* sdnn_version(void) { return "sdnn 0.1 (gfx950)"; }

sdnn_status sdnn_workspace_size(const sdnn_desc* desc, size_t* bytes) {
    TRY(check_desc(desc));
    if (!bytes) return fail(SDNN_EINVAL, "bytes is NULL");
    *bytes = make_layout(*desc).total;
    return SDNN_OK;
}

sdnn_status sdnn_ckpt_size(const sdnn_desc* desc, int64_t rows, size_t* bytes) {
    TRY(check_desc(desc));
    if (!bytes || rows < 0) return fail(SDNN_EINVAL, "bad arguments");
    const int S = desc->ckpt_every;
    if (S < 1) {
        *bytes = 0;
        return SDNN_OK;
    }
    const int64_t slots = (desc->n_layers + S - 1) / S - 1;
    *bytes = (size_t)std::max<int64_t>(slots, 0) * (size_t)rows * desc->n_neurons * 4;
    return SDNN_OK;
}

sdnn_status sdnn_create(const sdnn_desc* desc, const int32_t* idx, const float* w, const float* bias, void* workspace,
                        size_t ws_bytes, void* stream, sdnn_net* out) {
    TRY(check_desc(desc));
    if (!out) return fail(SDNN_EINVAL, "out is NULL");
    *out = nullptr;
    if (!idx || !w || !bias) return fail(SDNN_EINVAL, "idx, w and bias must be device pointers");
    if (((uintptr_t)idx | (uintptr_t)w) & 15) return fail(SDNN_EINVAL, "idx and w must be 16-byte aligned");
    const Layout lay = make_layout(*desc);
    if (!workspace) return fail(SDNN_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % ALIGN) return fail(SDNN_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < lay.total) return fail(SDNN_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, lay.total);
    hipStream_t s = (hipStream_t)stream;

    auto n = std::make_unique<sdnn_net_s>();
    n->d = *desc;
    n->idx = idx;
    n->w = w;
    n->b = bias;
    n->ws = (char*)workspace;
    n->ws_bytes = ws_bytes;
    n->lay = lay;
    n->act = (float*)(n->ws + lay.act);
    n->list0 = (int32_t*)(n->ws + lay.list0);
    n->list1 = (int32_t*)(n->ws + lay.list1);
    n->alive = (int32_t*)(n->ws + lay.alive);
    n->cnt = (int32_t*)(n->ws + lay.cnt);
    n->bar = (unsigned*)(n->ws + lay.bar);
    n->fin = (int32_t*)(n->ws + lay.fin);
    n->err = (int32_t*)(n->ws + lay.err);
    n->flag = (int32_t*)(n->ws + lay.flag);
    if (trainable(*desc)) {
        n->tr_ptr = (int32_t*)(n->ws + lay.tr_ptr);
        n->tr_e = (int32_t*)(n->ws + lay.tr_e);
        n->seg = (float*)(n->ws + lay.seg);
        n->gbuf0 = (float*)(n->ws + lay.gbuf0);
        n->gbuf1 = (float*)(n->ws + lay.gbuf1);
        n->pdw = (float*)(n->ws + lay.pdw);
        n->pdb = (float*)(n->ws + lay.pdb);
    }
    if (lay.wide) {
        n->wide = true;
        n->packed = (float*)(n->ws + lay.packed);
        n->wide_words = (int32_t*)(n->ws + lay.wide_words);
    }
    if (lay.row) {
        n->row = true;
        n->row_words = (int32_t*)(n->ws + lay.row_words);
        n->row_parts = row_parts(*desc);
    }
    if (lay.rowc) {
        n->row_words = (int32_t*)(n->ws + lay.row_words);
        n->row_parts = row_parts(*desc);
    }
    HIPCHK(hipGetDevice(&n->device));
    HIPCHK(hipDeviceGetAttribute(&n->num_cu, hipDeviceAttributeMultiprocessorCount, n->device));
    {
        void* h = nullptr;
        HIPCHK(hipHostMalloc(&h, 64, hipHostMallocMapped));
        n->herr = (int32_t*)h;
        *n->herr = 0;
        void* hd = nullptr;
        const hipError_t e = hipHostGetDevicePointer(&hd, h, 0);
        if (e != hipSuccess) {
            (void)hipHostFree(h);
            n->herr = nullptr;
            return fail(SDNN_EHIP, "hipHostGetDevicePointer failed: %s", hipGetErrorString(e));
        }
        n->herr_dev = (int32_t*)hd;
    }

    const int N = desc->n_neurons, L = desc->n_layers;
    const int64_t nnz = (int64_t)N * K * L;
    // error word, flags, barrier words
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, n->err, (int64_t)16, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, n->flag, (int64_t)16, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(2), dim3(256), 0, s, (int32_t*)n->bar, (int64_t)NBAR, 0);
    if (n->wide) {
        const int64_t nw = 2 * ((std::max<int64_t>(desc->max_rows, 1) + WIDE_TMIN - 1) / WIDE_TMIN);
        hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(nw)), dim3(256), 0, s, n->wide_words, nw, 0);
    }
    if (n->row_words) {
        const int64_t nw = std::max<int64_t>(desc->max_rows, 1);
        hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(nw)), dim3(256), 0, s, n->row_words, nw, 0);
    }
    HIPCHK(hipGetLastError());
    if (desc->flags & SDNN_DEBUG_CHECKS) {
        hipLaunchKernelGGL(k_check_params, dim3(blocks_for((int64_t)N * L)), dim3(256), 0, s, idx, w, bias, N, L,
                           n->flag, (float*)nullptr);
        HIPCHK(hipGetLastError());
        int32_t bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, n->flag, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (bad)
            return fail(SDNN_EINVAL, "parameter check failed:%s%s%s%s", (bad & 1) ? " idx out of range;" : "",
                        (bad & 2) ? " idx not strictly ascending;" : "", (bad & 4) ? " non-finite weight;" : "",
                        (bad & 8) ? " non-finite bias;" : "");
    }
    // Compaction is exact only while every bias is <= 0.
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, n->flag + 1, (int64_t)1, 0);
    hipLaunchKernelGGL(k_max_bias, dim3(blocks_for((int64_t)N * L)), dim3(256), 0, s, bias, (int64_t)N * L, n->flag + 1);
    HIPCHK(hipGetLastError());
    int32_t pos = 0;
    HIPCHK(hipMemcpyAsync(&pos, n->flag + 1, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    n->compaction = !(desc->flags & SDNN_NO_COMPACTION) && pos == 0;

    if (trainable(*desc)) {
        // transposed pattern per layer: counting sort of edge positions by input id
        int32_t* deg = (int32_t*)n->gbuf0;
        int32_t* cursor = deg + N;
        for (int l = 0; l < L; ++l) {
            const int32_t* il = idx + (size_t)l * N * K;
            int32_t* ptr = n->tr_ptr + (size_t)l * (N + 1);
            int32_t* te = n->tr_e + (size_t)l * N * K;
            hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(2 * N)), dim3(256), 0, s, deg, (int64_t)2 * N, 0);
            hipLaunchKernelGGL(k_tr_count, dim3(blocks_for((int64_t)N * K)), dim3(256), 0, s, il, (int64_t)N * K, deg);
            hipLaunchKernelGGL(k_tr_scan, dim3(1), dim3(1024), 0, s, (const int32_t*)deg, N, ptr);
            hipLaunchKernelGGL(k_tr_fill, dim3(blocks_for((int64_t)N * K)), dim3(256), 0, s, il, (int64_t)N * K,
                               (const int32_t*)ptr, cursor, te);
            hipLaunchKernelGGL(k_tr_sort, dim3(blocks_for(N)), dim3(256), 0, s, (const int32_t*)ptr, N, te);
        }
        HIPCHK(hipGetLastError());
        const size_t bsh = (size_t)bwd_T() * N * 4;
        HIPCHK(hipFuncSetAttribute(bwd_dw_fn(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bsh));
        HIPCHK(hipFuncSetAttribute(bwd_dy_fn(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bsh));
    }
    (void)nnz;
    if (lay.sched) {
        // slot schedule of every layer, built on the host from a copy of the ids
        n->nblk = (N + 63) / 64;
        n->parts = (n->nblk + 15) / 16;
        const size_t npad = (size_t)n->nblk * 64;
        n->ent = (uint32_t*)(n->ws + lay.ent);
        n->lane_neuron = (int32_t*)(n->ws + lay.lane_neuron);
        n->wave_steps = (int32_t*)(n->ws + lay.wave_steps);
        n->tile_bits = (int32_t*)(n->ws + lay.tile_bits);
        n->prog = (int32_t*)(n->ws + lay.prog);
        std::vector<int32_t> hidx((size_t)L * N * K);
        HIPCHK(hipMemcpyAsync(hidx.data(), idx, hidx.size() * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        bool ids_ok = true;
        for (size_t i = 0; i < hidx.size() && ids_ok; ++i) ids_ok = hidx[i] >= 0 && hidx[i] < N;
        if (ids_ok) {
            std::vector<uint32_t> hent((size_t)L * npad * SCHED_DSTORE);
            std::vector<int32_t> hln((size_t)L * npad), hws((size_t)L * n->nblk);
            const int worst = build_schedule(hidx.data(), N, L, SCHED_DSTORE, hent.data(), hln.data(), hws.data());
            if (worst <= SCHED_DSTORE) {
                // the kernel wants LDS byte offsets in buffer 0: id -> 2048 (id / 64) + 16 (id % 64)
                for (auto& e : hent) {
                    const uint32_t id = (e >> 5) & 0x03ffffffu;
                    e = (e & 0x8000001fu) | (sched_slot_offset(id) << 5);
                }
                // device layout is step-major per layer ([L][step][lane slot]): a wave's
                // 64 lanes read one step's entries with one coalesced load
                step_major(hent, L, npad);
                HIPCHK(hipMemcpyAsync(n->ent, hent.data(), hent.size() * 4, hipMemcpyHostToDevice, s));
                HIPCHK(hipMemcpyAsync(n->lane_neuron, hln.data(), hln.size() * 4, hipMemcpyHostToDevice, s));
                HIPCHK(hipMemcpyAsync(n->wave_steps, hws.data(), hws.size() * 4, hipMemcpyHostToDevice, s));
                const int64_t nt = (std::max<int64_t>(desc->max_rows, 1) + SCHED_T - 1) / SCHED_T;
                hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(nt)), dim3(256), 0, s, n->tile_bits, nt, 0);
                hipLaunchKernelGGL(k_fill_i32, dim3(4), dim3(256), 0, s, n->prog, (int64_t)SCHED_PROG, 0);
                HIPCHK(hipGetLastError());
                HIPCHK(hipStreamSynchronize(s));
                n->sched = true;
            }
            if (n->sched && trainable(*desc)) {
                // transposed schedule for the input-gradient gather: entries are edge
                // positions j*K + k; the kernel wants the LDS offset of column j and the edge
                std::vector<uint32_t> tent((size_t)L * npad * SCHED_DSTORE);
                std::vector<int32_t> tln((size_t)L * npad), tws((size_t)L * n->nblk);
                const int tworst =
                    build_transposed_schedule(hidx.data(), N, L, SCHED_DSTORE, tent.data(), tln.data(), tws.data());
                if (tworst <= SCHED_DSTORE) {
                    std::vector<uint32_t> tw(tent.size());
                    for (size_t i = 0; i < tent.size(); ++i) {
                        const uint32_t e = tent[i] & 0x7fffffffu;
                        const uint32_t col = e / K;
                        tw[i] = e;
                        tent[i] = (tent[i] & 0x80000000u) | (sched_slot_offset(col) << 5);
                    }
                    n->ent_t = (uint32_t*)(n->ws + lay.ent_t);
                    n->ent_w = (uint32_t*)(n->ws + lay.ent_w);
                    n->lane_input = (int32_t*)(n->ws + lay.lane_input);
                    n->steps_t = (int32_t*)(n->ws + lay.steps_t);
                    n->gbuf2 = (float*)(n->ws + lay.gbuf2);
                    step_major(tent, L, npad);
                    step_major(tw, L, npad);
                    HIPCHK(hipMemcpyAsync(n->ent_t, tent.data(), tent.size() * 4, hipMemcpyHostToDevice, s));
                    HIPCHK(hipMemcpyAsync(n->ent_w, tw.data(), tw.size() * 4, hipMemcpyHostToDevice, s));
                    HIPCHK(hipMemcpyAsync(n->lane_input, tln.data(), tln.size() * 4, hipMemcpyHostToDevice, s));
                    HIPCHK(hipMemcpyAsync(n->steps_t, tws.data(), tws.size() * 4, hipMemcpyHostToDevice, s));
                    HIPCHK(hipStreamSynchronize(s));
                    HIPCHK(hipFuncSetAttribute(bwd_dw_sched_fn(), hipFuncAttributeMaxDynamicSharedMemorySize,
                                              (int)sched_lds_bytes(N)));
                    HIPCHK(hipFuncSetAttribute(bwd_dy_sched_fn(), hipFuncAttributeMaxDynamicSharedMemorySize,
                                              (int)sched_lds_bytes(N)));
                    n->sched_bwd = true;
                }
            }
        }
    }
    if (lay.row_sched) {
        // bank-scheduled slot orders of the one-row-tile kernel, built on the host
        // from a copy of the ids (ids outside [0, N) leave the ascending order only)
        std::vector<int32_t> hidx((size_t)L * N * K);
        HIPCHK(hipMemcpyAsync(hidx.data(), idx, hidx.size() * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        bool ids_ok = true;
        for (size_t i = 0; i < hidx.size() && ids_ok; ++i) ids_ok = hidx[i] >= 0 && hidx[i] < N;
        if (ids_ok) {
            std::vector<uint8_t> perm((size_t)L * N * K);
            build_row_schedule(hidx.data(), N, L, perm.data());
            n->row_perm = (uint8_t*)(n->ws + lay.row_perm);
            HIPCHK(hipMemcpyAsync(n->row_perm, perm.data(), perm.size(), hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
        }
    }
    if (lay.rowc) {
        // the two-part kernel: whole pairs of parts and one weight value per layer (the
        // per-layer flags go through the activation buffer)
        bool uniform = false;
        if ((N / ROW_PART) % 2 == 0 && (size_t)L <= (size_t)std::max<int64_t>(desc->max_rows, 1) * N) {
            int32_t* flags = (int32_t*)n->act;
            hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(L)), dim3(256), 0, s, flags, (int64_t)L, 0);
            hipLaunchKernelGGL(k_weights_uniform, dim3(blocks_for(nnz)), dim3(256), 0, s, w, (int64_t)N * K, nnz, flags);
            HIPCHK(hipGetLastError());
            std::vector<int32_t> hf((size_t)L);
            HIPCHK(hipMemcpyAsync(hf.data(), flags, (size_t)L * 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            uniform = std::all_of(hf.begin(), hf.end(), [](int32_t f) { return f == 0; });
        }
        // neuron pairs of the chunked one-row-tile kernel, paired on the host from
        // per-neuron slot counts per chunk (computed on the device, max_rows layers at
        // a time through the activation buffer)
        const int C = rowc_chunks(*desc);
        std::vector<uint32_t> hcnt((size_t)L * N);
        const int64_t per = std::max<int64_t>(1, std::min<int64_t>(L, std::max<int64_t>(desc->max_rows, 1)));
        for (int64_t l0 = 0; l0 < L; l0 += per) {
            const int64_t nl = std::min<int64_t>(per, L - l0);
            hipLaunchKernelGGL(k_rowc_counts, dim3(blocks_for(nl * N)), dim3(256), 0, s, idx + (size_t)l0 * N * K,
                               nl * N, (int32_t)N, (int32_t)C, (uint32_t*)n->act);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(hcnt.data() + (size_t)l0 * N, n->act, (size_t)nl * N * 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        std::vector<uint32_t> pairs((size_t)L * N / 2);
        const int worst = build_rowc_pairs(hcnt.data(), N, L, C, pairs.data());
        if (worst >= 0 && worst <= ROWC_OVF_CAP) {
            // the lane images, built on the device from the pairs (uploaded through the
            // activation buffer, 2 max_rows layers at a time)
            n->rowc_img = (uint32_t*)(n->ws + lay.rowc_img);
            n->rowc_meta = (uint32_t*)(n->ws + lay.rowc_meta);
            n->rowc_ovf = (uint32_t*)(n->ws + lay.rowc_ovf);
            const int G = N / ROW_PART;
            const int64_t per2 = std::max<int64_t>(1, std::min<int64_t>({(int64_t)L, 2 * std::max<int64_t>(desc->max_rows, 1),
                                                                       (int64_t)65535}));
            int32_t* status = n->flag + 3;                 // [0] a list overflowed, [1] longest list
            hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, status, (int64_t)2, 0);
            for (int64_t l0 = 0; l0 < L; l0 += per2) {
                const int64_t nl = std::min<int64_t>(per2, L - l0);
                HIPCHK(hipMemcpyAsync(n->act, pairs.data() + (size_t)l0 * N / 2, (size_t)nl * N / 2 * 4,
                                      hipMemcpyHostToDevice, s));
                const size_t lp = (size_t)l0 * G;
                hipLaunchKernelGGL(k_rowc_build, dim3(G, (unsigned)nl), dim3(ROW_NT), 0, s, idx + (size_t)l0 * N * K,
                                   w + (size_t)l0 * N * K, (const uint32_t*)n->act, (int32_t)N, (int32_t)C,
                                   (int32_t)(uniform ? RU_ZERO : 0),
                                   n->rowc_img + lp * ROWC_IMG * ROW_NT, n->rowc_meta + lp * ROW_NT * 4,
                                   n->rowc_ovf + lp * ROWC_OVF_CAP * 2, status);
                HIPCHK(hipGetLastError());
                HIPCHK(hipStreamSynchronize(s));
            }
            // the bank order of every (layer, part, half-wave block)
            const int64_t tasks = (int64_t)L * G * 32;
            hipLaunchKernelGGL(k_rowc_sched, dim3((unsigned)std::min<int64_t>(4096, (tasks + 63) / 64)), dim3(64), 0, s,
                               n->rowc_img, n->rowc_meta, tasks, (int32_t)C);
            HIPCHK(hipGetLastError());
            int32_t st[2] = {0, 0};
            HIPCHK(hipMemcpyAsync(st, status, 8, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            n->rowc = st[0] == 0;
            n->rowc_chunks = C;
            if (n->rowc && uniform && st[1] <= RU_OVF_CAP) {
                // padding reads the zero words at the end of the two-part kernel's buffers
                const int64_t lanes = (int64_t)L * G * ROW_NT;
                hipLaunchKernelGGL(k_rowu_pads, dim3(blocks_for(lanes)), dim3(256), 0, s, n->rowc_img, lanes,
                                   (uint32_t)(4 * (N / C - RU_ZERO)));
                HIPCHK(hipGetLastError());
                HIPCHK(hipStreamSynchronize(s));
                n->rowu = true;
            }
        }
    }
    n->variant = default_variant(n.get());
    TRY(prepare_variant(n.get(), n->variant, &n->grid, &n->chain_grid));
    HIPCHK(hipStreamSynchronize(s));
    sdnn_net net = n.release();
    if (desc->flags & SDNN_AUTOTUNE) {
        const sdnn_status st = sdnn_tune(net, nullptr, desc->max_rows, stream);
        if (st != SDNN_OK) {
            sdnn_destroy(net);
            return st;
        }
    }
    *out = net;
    return SDNN_OK;
}

sdnn_status sdnn_set_exec(sdnn_net net, int32_t mode) {
    if (!net) return fail(SDNN_EINVAL, "net is NULL");
    if (mode < SDNN_EXEC_AUTO || mode > SDNN_EXEC_GRAPH_MERGED) return fail(SDNN_EINVAL, "unknown exec mode %d", mode);
    net->exec = mode;
    return SDNN_OK;
}

sdnn_status sdnn_set_timing(sdnn_net net, int32_t enable) {
    if (!net) return fail(SDNN_EINVAL, "net is NULL");
    net->timing = enable != 0;
    return SDNN_OK;
}

sdnn_status sdnn_kernel_time(sdnn_net net, double* total_ms, int32_t* launches) {
    if (!net) return fail(SDNN_EINVAL, "net is NULL");
    double tot = 0.0;
    for (size_t i = 0; i + 1 < net->tev_used; i += 2) {
        HIPCHK(hipEventSynchronize(net->tev[i + 1]));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, net->tev[i], net->tev[i + 1]));
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = (int32_t)(net->tev_used / 2);
    net->tev_used = 0;
    return SDNN_OK;
}

sdnn_status sdnn_get_plan(sdnn_net net, sdnn_plan* plan) {
    if (!net || !plan) return fail(SDNN_EINVAL, "NULL argument");
    const FwdVariant& v = var(net);
    plan->rows_per_tile = v.T;
    plan->threads = v.NT;
    plan->grid = net->grid;
    plan->variant = v.staged >= 2 ? v.staged : (v.staged ? 0 : 1);
    plan->tuned_us = net->tuned_us;
    return SDNN_OK;
}

sdnn_status sdnn_set_plan(sdnn_net net, const sdnn_plan* plan) {
    if (!net || !plan) return fail(SDNN_EINVAL, "NULL argument");
    for (int vi = 0; vi < fwd_variant_count(); ++vi) {
        const FwdVariant& v = fwd_variant(vi);
        const int code = v.staged >= 2 ? v.staged : (v.staged ? 0 : 1);
        if (v.T != plan->rows_per_tile || v.NT != plan->threads || code != plan->variant) continue;
        if (!variant_fits(net, v))
            return fail(SDNN_EUNSUPPORTED, "variant %d (T=%d, NT=%d) does not fit this net", code, v.T, v.NT);
        int g = 0, cg = 0;
        TRY(prepare_variant(net, vi, &g, &cg));
        net->variant = vi;
        net->grid = g;
        net->chain_grid = cg;
        drop_graph(net);
        return SDNN_OK;
    }
    return fail(SDNN_EINVAL, "no kernel variant with T=%d, NT=%d, variant=%d", plan->rows_per_tile, plan->threads,
                plan->variant);
}

sdnn_status sdnn_tune(sdnn_net net, const float* y_sample, int64_t rows, void* stream) {
    if (!net) return fail(SDNN_EINVAL, "net is NULL");
    TRY(host_error(net));
    if (rows < 0) return fail(SDNN_EINVAL, "rows < 0");
    if (y_sample && rows > net->d.max_rows)
        return fail(SDNN_EINVAL, "rows = %lld exceeds max_rows = %lld", (long long)rows, (long long)net->d.max_rows);
    hipStream_t s = (hipStream_t)stream;
    const int N = net->d.n_neurons;
    // the caller's rows (outputs into the workspace buffer), or all-ones rows in the
    // first half of the workspace buffer and the outputs in its second half
    const int64_t rt = y_sample ? rows : std::min<int64_t>(rows, net->d.max_rows / 2);
    if (rt < 1) return SDNN_OK;   // nothing to time with
    const float* in = y_sample ? y_sample : net->act;
    float* outb = y_sample ? net->act : net->act + (size_t)rt * N;
    if (!y_sample) {
        hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for(rt * N)), dim3(256), 0, s, net->act, rt * N, 1.0f);
        HIPCHK(hipGetLastError());
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best = 1e30f;
    int best_v = net->variant, best_g = net->grid, best_cg = net->chain_grid;
    // The kernel that matters is the one the forward runs: the persistent chain
    // kernel (timed here over one layer: init, then the cooperative launch with its
    // work list, liveness and grid barrier), or, for the graph and eager forms, the
    // per-layer launch.
    const bool chain = net->exec == SDNN_EXEC_PERSISTENT || net->exec == SDNN_EXEC_AUTO;
    // Variants of one family share the per-output arithmetic order (the scheduled
    // kernels sum slots in their create-time order), so tuning never changes results.
    auto family = [](int staged) { return staged == 2 || staged == 5 || staged == 6 || staged == 7 ? staged : 0; };
    const int fam = family(var(net).staged);
    for (int vi = 0; vi < fwd_variant_count(); ++vi) {
        const FwdVariant& v = fwd_variant(vi);
        if (!variant_fits(net, v) || family(v.staged) != fam) continue;
        int g = 0, cg = 0;
        if (prepare_variant(net, vi, &g, &cg) != SDNN_OK) continue;
        std::unique_ptr<Launch> init, run;
        if (chain) {
            // a one-layer chain: layer 0 reads `in` and writes `outb` (its output buffer)
            ChainArgs c{};
            c.y0 = in;
            c.y_out = outb;
            c.act = outb;
            c.idx = net->idx;
            c.w = net->w;
            c.b = net->b;
            c.list0 = net->list0;
            c.list1 = net->list1;
            c.cnt = net->cnt;
            c.alive = net->alive;
            c.bar = net->bar;
            c.err = net->err;
            c.rows = (int32_t)rt;
            c.N = N;
            c.L = 1;
            c.ckpt_every = 2;
            c.compaction = net->compaction ? 1 : 0;
            c.clamp = net->d.clamp;
            if (net->sched) {
                c.ent = net->ent;
                c.lane_neuron = net->lane_neuron;
                c.wave_steps = net->wave_steps;
                c.tile_bits = net->tile_bits;
                c.prog = net->prog;
                c.parts = net->parts;
                c.nblk = net->nblk;
            }
            c.packed = net->packed;
            c.wide_words = net->wide_words;
            c.row_words = net->row_words;
            c.row_parts = net->row_parts;
            c.row_perm = net->row_perm;
            c.rowc_img = net->rowc_img;
            c.rowc_meta = net->rowc_meta;
            c.rowc_ovf = net->rowc_ovf;
            init = mk((const void*)&k_chain_init, dim3(1), dim3(256), 0, net->cnt, (int32_t)1, (int32_t)rt,
                      (int32_t)c.compaction, net->bar, (int32_t)NBAR);
            run = mk(v.chain_fn, dim3(cg), dim3(v.NT), fwd_lds_bytes(v, N), c);
            run->cooperative = true;
        }
        LayerArgs a{};
        a.yin = in;
        a.yout = outb;
        a.idx = net->idx;
        a.w = net->w;
        a.b = net->b;
        a.nrows = (int32_t)rt;
        a.N = N;
        a.clamp = net->d.clamp;
        fill_sched(net, a, 0);
        const int gg = v.staged >= 2 ? g : std::max(1, std::min<int>(g, (int)((rt + v.T - 1) / v.T)));
        auto once = [&]() -> sdnn_status {
            if (!chain) {
                HIPCHK(launch_layer(net, v, gg, a, rt, s));
                return SDNN_OK;
            }
            Plan p;
            p.push_back(std::move(init));
            p.push_back(std::move(run));
            const sdnn_status st = issue(p, s);
            init = std::move(p[0]);
            run = std::move(p[1]);
            return st;
        };
        TRY(once());
        HIPCHK(hipEventRecord(e0, s));
        const int reps = 3;
        for (int r = 0; r < reps; ++r) TRY(once());
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        const float us = ms * 1000.f / reps;
        if (us < best) {
            best = us;
            best_v = vi;
            best_g = g;
            best_cg = cg;
        }
    }
    HIPCHK(hipEventDestroy(e0));
    HIPCHK(hipEventDestroy(e1));
    net->variant = best_v;
    net->grid = best_g;
    net->chain_grid = best_cg;
    net->tuned_us = best < 1e29f ? best : 0.f;
    drop_graph(net);
    return SDNN_OK;
}

sdnn_status sdnn_forward(sdnn_net net, const float* y0, int64_t rows, const int64_t* batch_off, int32_t n_batches,
                         float* y_out, int32_t* nz_rows, int32_t* n_nz, float* ckpt, int32_t* layer_rows,
                         void* stream) {
    if (!net) return fail(SDNN_EINVAL, "net is NULL");
    TRY(host_error(net));
    const sdnn_desc& d = net->d;
    if (rows < 0 || rows > d.max_rows) return fail(SDNN_EINVAL, "rows = %lld outside [0, max_rows = %lld]",
                                                  (long long)rows, (long long)d.max_rows);
    if (!n_nz || !nz_rows) return fail(SDNN_EINVAL, "nz_rows and n_nz are required");
    if (rows > 0 && (!y0 || !y_out)) return fail(SDNN_EINVAL, "y0 and y_out are required");
    const size_t bytes = (size_t)rows * d.n_neurons * 4;
    if (rows > 0 && (const char*)y0 < (const char*)y_out + bytes && (const char*)y_out < (const char*)y0 + bytes)
        return fail(SDNN_EINVAL, "y0 and y_out overlap");
    if (ckpt && d.ckpt_every < 1) return fail(SDNN_EINVAL, "ckpt given but the net has ckpt_every = 0");
    std::vector<int64_t> off;
    if (batch_off) {
        if (n_batches < 1 || n_batches > MAX_BATCHES)
            return fail(SDNN_EINVAL, "n_batches = %d outside [1, %d]", n_batches, MAX_BATCHES);
        off.assign(batch_off, batch_off + n_batches + 1);
        if (off[0] != 0 || off[n_batches] != rows) return fail(SDNN_EINVAL, "batch offsets must run from 0 to rows");
        for (int i = 0; i < n_batches; ++i)
            if (off[i + 1] < off[i]) return fail(SDNN_EINVAL, "batch offsets must be non-decreasing");
    } else {
        off = {0, rows};
        n_batches = 1;
    }
    hipStream_t s = (hipStream_t)stream;
    const int L = d.n_layers;
    if (rows == 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, n_nz, (int64_t)1, 0);
        if (layer_rows) hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(L + 1)), dim3(256), 0, s, layer_rows, (int64_t)L + 1, 0);
        HIPCHK(hipGetLastError());
        return SDNN_OK;
    }
    int mode = net->exec;
    // the wide-layer kernels take two graph nodes per layer (pack, compute), empty
    // layers included; their persistent chain skips the empty ones (C4: 28.8 against
    // 40.6 ms for the merged graph); the chunked one-row-tile kernel's layers load
    // their lane images first, so its persistent chain also wins on the deep nets
    // (C4: 20.6 against 26 ms)
    if (mode == SDNN_EXEC_AUTO)
        mode = (var(net).staged == 3 || var(net).staged == 6 || var(net).staged == 7)
                   ? SDNN_EXEC_PERSISTENT
                   : (n_batches > 1 ? SDNN_EXEC_GRAPH_MERGED : SDNN_EXEC_GRAPH);
    if (mode == SDNN_EXEC_PERSISTENT) {
        Plan p = plan_persistent(net, y0, rows, y_out, nz_rows, n_nz, ckpt, layer_rows);
        return issue(p, s, net);
    }
    // GRAPH / EAGER: batches one after another; GRAPH_MERGED: one chain over all rows.
    const bool merged = mode == SDNN_EXEC_GRAPH_MERGED;
    if (mode == SDNN_EXEC_EAGER) {
        Plan p = merged ? plan_merged(net, y0, rows, y_out, nz_rows, n_nz, ckpt, layer_rows)
                        : plan_chain(net, y0, rows, off.data(), n_batches, y_out, nz_rows, n_nz, ckpt, layer_rows);
        return issue(p, s);
    }
    std::vector<int64_t> key = {(int64_t)(uintptr_t)y0, (int64_t)(uintptr_t)y_out, (int64_t)(uintptr_t)nz_rows,
                                (int64_t)(uintptr_t)n_nz, (int64_t)(uintptr_t)ckpt, (int64_t)(uintptr_t)layer_rows,
                                rows, net->variant, net->grid, merged ? 1 : 0};
    key.insert(key.end(), off.begin(), off.end());
    if (!net->gexec || key != net->gkey) {
        Plan p = merged ? plan_merged(net, y0, rows, y_out, nz_rows, n_nz, ckpt, layer_rows)
                        : plan_chain(net, y0, rows, off.data(), n_batches, y_out, nz_rows, n_nz, ckpt, layer_rows);
        TRY(build_graph(net, p));
        net->gkey = key;
    }
    HIPCHK(hipGraphLaunch(net->gexec, s));
    return SDNN_OK;
}

sdnn_status sdnn_layer(sdnn_net net, int32_t layer, const float* y_in, int64_t rows, float* y_out, void* stream) {
    if (!net) return fail(SDNN_EINVAL, "net is NULL");
    TRY(host_error(net));
    const sdnn_desc& d = net->d;
    if (layer < 0 || layer >= d.n_layers) return fail(SDNN_EINVAL, "layer %d out of range", layer);
    if (rows < 0 || rows > d.max_rows) return fail(SDNN_EINVAL, "rows = %lld outside [0, max_rows = %lld]",
                                                  (long long)rows, (long long)d.max_rows);
    if (rows == 0) return SDNN_OK;
    if (!y_in || !y_out) return fail(SDNN_EINVAL, "y_in and y_out are required");
    const size_t bytes = (size_t)rows * d.n_neurons * 4;
    if ((const char*)y_in < (const char*)y_out + bytes && (const char*)y_out < (const char*)y_in + bytes)
        return fail(SDNN_EINVAL, "y_in and y_out overlap");
    const FwdVariant& v = var(net);
    const size_t NK = (size_t)d.n_neurons * K;
    LayerArgs a{};
    a.yin = y_in;
    a.yout = y_out;
    a.idx = net->idx + layer * NK;
    a.w = net->w + layer * NK;
    a.b = net->b + (size_t)layer * d.n_neurons;
    a.nrows = (int32_t)rows;
    a.N = d.n_neurons;
    a.layer = layer;
    a.clamp = d.clamp;
    fill_sched(net, a, layer);
    HIPCHK(launch_layer(net, v, launch_grid(net, v, rows), a, rows, (hipStream_t)stream));
    return SDNN_OK;
}

sdnn_status sdnn_backward(sdnn_net net, const float* y0, int64_t rows, const float* ckpt, const int32_t* nz_rows,
                          const int32_t* n_nz, const float* dy_out, float* dw, float* dbias, float* dy0,
                          void* stream) {
    if (!net) return fail(SDNN_EINVAL, "net is NULL");
    TRY(host_error(net));
    const sdnn_desc& d = net->d;
    if (!trainable(d)) return fail(SDNN_EINVAL, "net was not created with SDNN_TRAINABLE");
    if (rows < 0 || rows > d.max_rows) return fail(SDNN_EINVAL, "rows out of range");
    if (!nz_rows || !n_nz || !dw || !dbias) return fail(SDNN_EINVAL, "nz_rows, n_nz, dw and dbias are required");
    const int L = d.n_layers, N = d.n_neurons, S = d.ckpt_every;
    const int nseg = (L + S - 1) / S;
    if (rows > 0 && (!y0 || !dy_out)) return fail(SDNN_EINVAL, "y0 and dy_out are required");
    if (rows > 0 && nseg > 1 && !ckpt) return fail(SDNN_EINVAL, "ckpt is required when n_layers > ckpt_every");
    hipStream_t s = (hipStream_t)stream;
    const size_t NK = (size_t)N * K;
    if (dy0) {
        hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for((int64_t)rows * N)), dim3(256), 0, s, dy0, (int64_t)rows * N, 0.f);
    }
    if (rows == 0) {
        hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for((int64_t)L * NK)), dim3(256), 0, s, dw, (int64_t)L * NK, 0.f);
        hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for((int64_t)L * N)), dim3(256), 0, s, dbias, (int64_t)L * N, 0.f);
        HIPCHK(hipGetLastError());
        return SDNN_OK;
    }
    const size_t RN = (size_t)d.max_rows * N;
    auto seg = [&](int i) { return net->seg + (size_t)i * RN; };
    float* D = net->gbuf0;
    float* Dn = net->gbuf1;
    const int gather_grid = std::min<int64_t>(rows, 8192);
    hipLaunchKernelGGL(k_gather_rows, dim3(gather_grid), dim3(256), 0, s, dy_out, nz_rows, n_nz, N, D);
    const FwdVariant& v = var(net);
    const int fgrid = launch_grid(net, v, rows);
    const size_t bsh = (size_t)bwd_T() * N * 4;
    const int dy_grid = std::max(1, std::min<int>(net->num_cu * 2, (int)((rows + bwd_T() - 1) / bwd_T())));
    for (int sg = nseg - 1; sg >= 0; --sg) {
        const int l0 = sg * S, l1 = std::min(L, l0 + S);
        const float* src = sg == 0 ? y0 : ckpt + (size_t)(sg - 1) * rows * N;
        hipLaunchKernelGGL(k_gather_rows, dim3(gather_grid), dim3(256), 0, s, src, nz_rows, n_nz, N, seg(0));
        for (int l = l0; l < l1; ++l) {
            LayerArgs a{};
            a.yin = seg(l - l0);
            a.yout = seg(l - l0 + 1);
            a.idx = net->idx + l * NK;
            a.w = net->w + l * NK;
            a.b = net->b + (size_t)l * N;
            a.cnt_in = n_nz;
            a.N = N;
            a.layer = l;
            a.clamp = d.clamp;
            fill_sched(net, a, l);
            HIPCHK(launch_layer(net, v, fgrid, a, rows, s));
        }
        for (int l = l1 - 1; l >= l0; --l) {
            const bool sch = net->sched_bwd && var(net).staged == 2;
            if (sch) {
                TRY(backward_layer_sched(net, l, seg(l - l0), seg(l - l0 + 1), D, (l > 0 || dy0) ? (l == 0 ? dy0 : Dn) : nullptr,
                                         l == 0 ? nz_rows : nullptr, n_nz, rows, dw + (size_t)l * NK,
                                         dbias + (size_t)l * N, s));
                if (l > 0 || dy0) std::swap(D, Dn);
                continue;
            }
            BwdDwArgs da{};
            da.y_in = seg(l - l0);
            da.y_out = seg(l - l0 + 1);
            da.dy = D;
            da.idx = net->idx + l * NK;
            da.nrows = n_nz;
            da.pdw = net->pdw;
            da.pdb = net->pdb;
            da.N = N;
            da.P = P_GROUPS;
            da.clamp = d.clamp;
            void* dargs[] = {&da};
            HIPCHK(hipLaunchKernel(bwd_dw_fn(), dim3(P_GROUPS, (N + bwd_threads() - 1) / bwd_threads()),
                                   dim3(bwd_threads()), dargs, bsh, s));
            hipLaunchKernelGGL(k_reduce_partials, dim3(blocks_for((int64_t)NK + N)), dim3(256), 0, s,
                               (const float*)net->pdw, (const float*)net->pdb, (int32_t)P_GROUPS, (int32_t)N,
                               dw + (size_t)l * NK, dbias + (size_t)l * N, (const int32_t*)nullptr, (int32_t)1);
            if (l > 0 || dy0) {
                BwdDyArgs ya{};
                ya.y_out = seg(l - l0 + 1);
                ya.dy = D;
                ya.tr_ptr = net->tr_ptr + (size_t)l * (N + 1);
                ya.tr_e = net->tr_e + (size_t)l * NK;
                ya.w = net->w + l * NK;
                ya.nrows = n_nz;
                ya.rows_out = l == 0 ? nz_rows : nullptr;
                ya.dy_in = l == 0 ? dy0 : Dn;
                ya.N = N;
                ya.clamp = d.clamp;
                void* yargs[] = {&ya};
                HIPCHK(hipLaunchKernel(bwd_dy_fn(), dim3(dy_grid), dim3(bwd_threads()), yargs, bsh, s));
                std::swap(D, Dn);
            }
        }
    }
    HIPCHK(hipGetLastError());
    return SDNN_OK;
}

sdnn_status sdnn_layer_backward(sdnn_net net, int32_t layer, const float* y_in, const float* y_out,
                                const float* dy_out, int64_t rows, float* dw, float* dbias, float* dy_in,
                                void* stream) {
    if (!net) return fail(SDNN_EINVAL, "net is NULL");
    TRY(host_error(net));
    const sdnn_desc& d = net->d;
    if (!trainable(d)) return fail(SDNN_EINVAL, "net was not created with SDNN_TRAINABLE");
    if (layer < 0 || layer >= d.n_layers) return fail(SDNN_EINVAL, "layer %d out of range", layer);
    if (rows < 0 || rows > d.max_rows) return fail(SDNN_EINVAL, "rows out of range");
    if (!dw || !dbias) return fail(SDNN_EINVAL, "dw and dbias are required");
    if (rows > 0 && (!y_in || !y_out || !dy_out)) return fail(SDNN_EINVAL, "y_in, y_out and dy_out are required");
    hipStream_t s = (hipStream_t)stream;
    const int N = d.n_neurons;
    const size_t NK = (size_t)N * K;
    int32_t* nrows = net->flag + 2;                      // device copy of `rows`
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, nrows, (int64_t)1, (int32_t)rows);
    if (net->sched_bwd && var(net).staged == 2)
        return backward_layer_sched(net, layer, y_in, y_out, dy_out, rows > 0 ? dy_in : nullptr, nullptr, nrows, rows,
                                    dw, dbias, s);
    const size_t bsh = (size_t)bwd_T() * N * 4;
    BwdDwArgs da{};
    da.y_in = y_in;
    da.y_out = y_out;
    da.dy = dy_out;
    da.idx = net->idx + layer * NK;
    da.nrows = nrows;
    da.pdw = net->pdw;
    da.pdb = net->pdb;
    da.N = N;
    da.P = P_GROUPS;
    da.clamp = d.clamp;
    void* dargs[] = {&da};
    HIPCHK(hipLaunchKernel(bwd_dw_fn(), dim3(P_GROUPS, (N + bwd_threads() - 1) / bwd_threads()), dim3(bwd_threads()),
                           dargs, bsh, s));
    hipLaunchKernelGGL(k_reduce_partials, dim3(blocks_for((int64_t)NK + N)), dim3(256), 0, s, (const float*)net->pdw,
                       (const float*)net->pdb, (int32_t)P_GROUPS, (int32_t)N, dw, dbias, (const int32_t*)nullptr,
                       (int32_t)1);
    if (dy_in && rows > 0) {
        BwdDyArgs ya{};
        ya.y_out = y_out;
        ya.dy = dy_out;
        ya.tr_ptr = net->tr_ptr + (size_t)layer * (N + 1);
        ya.tr_e = net->tr_e + (size_t)layer * NK;
        ya.w = net->w + layer * NK;
        ya.nrows = nrows;
        ya.rows_out = nullptr;
        ya.dy_in = dy_in;
        ya.N = N;
        ya.clamp = d.clamp;
        void* yargs[] = {&ya};
        const int g = std::max(1, std::min<int>(net->num_cu * 2, (int)((rows + bwd_T() - 1) / bwd_T())));
        HIPCHK(hipLaunchKernel(bwd_dy_fn(), dim3(g), dim3(bwd_threads()), yargs, bsh, s));
    }
    HIPCHK(hipGetLastError());
    return SDNN_OK;
}

sdnn_status sdnn_mse(const float* y, const float* t, int64_t n, float* dy, float* loss, void* stream) {
    if (n < 0) return fail(SDNN_EINVAL, "n < 0");
    if (n > 0 && (!y || !t)) return fail(SDNN_EINVAL, "y and t are required");
    if (!dy && !loss) return SDNN_OK;
    hipStream_t s = (hipStream_t)stream;
    // loss[1 .. MSE_BLOCKS] are scratch for the per-block partial sums
    float* partial = loss ? loss + 1 : nullptr;
    if (!loss) {
        hipLaunchKernelGGL(k_mse, dim3(MSE_BLOCKS), dim3(256), 0, s, y, t, n, dy, (float*)nullptr, n ? 2.f / (float)n : 0.f);
    } else {
        hipLaunchKernelGGL(k_mse, dim3(MSE_BLOCKS), dim3(256), 0, s, y, t, n, dy, partial, n ? 2.f / (float)n : 0.f);
        hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, s, (const float*)partial, (int32_t)MSE_BLOCKS, loss,
                           n ? 1.f / (float)n : 0.f);
    }
    HIPCHK(hipGetLastError());
    return SDNN_OK;
}

// ---------------------------------------------------------------- no-allocation MSE
// sdnn_mse_noalloc keeps the per-workgroup partial sums in this file-scope device
// array (each GPU the library runs on holds its own copy until the process ends)
// instead of the caller's loss[1 .. MSE_BLOCKS].  Host code never passes the
// array's name to a kernel: it is a host-side stand-in, not a device address.  The
// device address comes from hipGetSymbolAddress, once per device, on the first call.
constexpr int MSE_SCRATCH_FLOATS = 256;
static_assert(MSE_BLOCKS <= MSE_SCRATCH_FLOATS, "the MSE partial sums must fit the static scratch");
static __device__ __align__(256) float scratch[MSE_SCRATCH_FLOATS];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[SCRATCH_MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on first use).
sdnn_status scratch_address(float** out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
        return fail(SDNN_EUNSUPPORTED, "device ordinal %d is beyond the %d devices the static scratch serves", dev,
                    SCRATCH_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SDNN_EHIP, "hipGetSymbolAddress returned NULL for the MSE scratch on device %d", dev);
        g_scratch_dev[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_dev[dev];
    return SDNN_OK;
}
}  // namespace

sdnn_status sdnn_mse_noalloc(const float* y, const float* t, int64_t n, float* dy, float* loss, void* stream) {
    if (n < 0) return fail(SDNN_EINVAL, "n < 0");
    if (n > 0 && (!y || !t)) return fail(SDNN_EINVAL, "y and t are required");
    if (!dy && !loss) return SDNN_OK;
    hipStream_t s = (hipStream_t)stream;
    float* partial = nullptr;
    if (loss) TRY(scratch_address(&partial));
    // the same two kernels as sdnn_mse, so results are bitwise equal to it; every
    // workgroup of k_mse writes its partial, so the scratch needs no clearing
    hipLaunchKernelGGL(k_mse, dim3(MSE_BLOCKS), dim3(256), 0, s, y, t, n, dy, partial, n ? 2.f / (float)n : 0.f);
    if (loss)
        hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, s, (const float*)partial, (int32_t)MSE_BLOCKS, loss,
                           n ? 1.f / (float)n : 0.f);
    HIPCHK(hipGetLastError());
    return SDNN_OK;
}

int64_t sdnn_row_schedule_host(const int32_t* idx, int32_t n_neurons, int32_t n_layers, uint8_t* perm) {
    if (!idx || !perm || n_neurons < K || n_layers < 1) return fail(SDNN_EINVAL, "bad arguments");
    for (size_t i = 0; i < (size_t)n_layers * n_neurons * K; ++i)
        if (idx[i] < 0 || idx[i] >= n_neurons) return fail(SDNN_EINVAL, "idx out of range");
    return build_row_schedule(idx, n_neurons, n_layers, perm);
}

int32_t sdnn_schedule_host(const int32_t* idx, int32_t n_neurons, int32_t n_layers, int32_t dmax, uint32_t* ent,
                           int32_t* lane_neuron, int32_t* steps) {
    if (!idx || !ent || !lane_neuron || !steps || n_neurons < K || n_layers < 1 || dmax < K)
        return fail(SDNN_EINVAL, "bad arguments");
    for (size_t i = 0; i < (size_t)n_neurons * n_layers * K; ++i)
        if (idx[i] < 0 || idx[i] >= n_neurons) return fail(SDNN_EINVAL, "id out of range");
    return build_schedule(idx, n_neurons, n_layers, dmax, ent, lane_neuron, steps);
}

sdnn_status sdnn_check_device(sdnn_net net, void* stream) {
    if (!net) return fail(SDNN_EINVAL, "net is NULL");
    hipStream_t s = (hipStream_t)stream;
    int32_t e = 0;
    HIPCHK(hipMemcpyAsync(&e, net->err, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (e != 0 && net->herr) __atomic_store_n(net->herr, e, __ATOMIC_RELEASE);
    if (e == DEV_BARRIER_TIMEOUT) return fail(SDNN_EDEVICE, "a persistent-kernel grid barrier timed out");
    if (e != 0) return fail(SDNN_EDEVICE, "device error %d", e);
    return SDNN_OK;
}

sdnn_status sdnn_inject_device_error(sdnn_net net, int32_t code, void* stream) {
    if (!net) return fail(SDNN_EINVAL, "net is NULL");
    if (code == 0) return fail(SDNN_EINVAL, "code must be nonzero");
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, (hipStream_t)stream, net->err, (int64_t)1, code);
    HIPCHK(hipGetLastError());
    return SDNN_OK;
}

void sdnn_destroy(sdnn_net net) {
    if (!net) return;
    drop_graph(net);
    for (hipEvent_t e : net->tev) (void)hipEventDestroy(e);
    net->tev.clear();
    delete net;
}

}  // extern "C"
