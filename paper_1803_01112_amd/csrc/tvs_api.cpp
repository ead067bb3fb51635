// tvs_api.cpp -- the C ABI (include/tvs.h) and the host runtime around the
// gfx950 kernels: argument validation, device memory ownership and HBM
// budget, history ingest and the tile lists of every DROP block (their
// layout fixed at load; rows formed once for a path store, per chunk and
// sweep for on-the-fly rows), the cycle driver (schedule of ell and beta,
// TV steps with or without the TV-reduction check, the DROP sweep) and the
// step log.
//
// Cycle structure (arXiv 1803.01112, Appendix C): ell_k = rand(k, ell_{k-1})
// once per cycle; N perturbation steps with beta = alpha^ell, ell += 1 after
// each; then x = P_T(x).  With the check, each step retries z = x + beta v
// with ell += 1 (and beta = alpha^ell recomputed) until TV(z) <= TV(x).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tvs_internal.hpp"

using tvs::GridDev;
using tvs::HistDev;
using tvs::RowSet;
using tvs::TileBlock;

namespace {

constexpr int kNumStreams = 13;
constexpr uint32_t kTileShiftHost = (uint32_t)tvs::kTileShift;

// Step records of checked cycles held on the device before they are copied
// back (once per call, or when the buffer fills).
constexpr int64_t kDevLogCap = 4096;

// On the fly, rows are formed into a ring of chunk buffers: with three, the
// formation stream can form the next sweep's first chunk while the DROP
// chain still reads the last two of this sweep.
constexpr int kChunkBuffers = 3;

// Flags on the device: DROP fixed-point range, tile-list consistency,
// history validation, longest vertex count, longest chord (float32 bits).
enum {
    kFlagRange = 0,
    kFlagLists = 1,
    kFlagInvalid = 2,
    kFlagJmax = 3,
    kFlagChordMax = 4,
    kNumFlags = 5
};

// SplitMix64 (Steele, Lea, Flood 2014): golden-gamma Weyl state, variant-13
// output mixer.
uint64_t splitmix64(uint64_t &state)
{
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// rand(k, ell): uniform integer in [k, ell], both ends included (k when
// ell < k); exactly one draw per call.
int64_t draw_ell(int64_t k, int64_t ell, uint64_t &state)
{
    uint64_t u = splitmix64(state);
    if (ell < k) return k;
    uint64_t span = (uint64_t)(ell - k) + 1u;
    unsigned __int128 p = (unsigned __int128)u * span;
    return k + (int64_t)(uint64_t)(p >> 64);
}

// Device workspace of tvs_initial_fbp_noalloc: one file-scope array, held by
// every device the library runs on until the process ends.  Host code never
// uses the array's name as an address: each device's copy is looked up once
// (fbp_scratch_setup, from tvs_create with that device current) and its
// address is passed to the kernels.
constexpr size_t kFbpScratchBytes = (size_t)64 << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kFbpScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_status[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Looks up this device's copy of `scratch` (the device must be current).
void fbp_scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_done[dev]) return;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    g_scratch_ptr[dev] = p;
    g_scratch_status[dev] = e;
    g_scratch_done[dev] = true;
}

}  // namespace

struct tvs_ctx {
    tvs_grid grid{};
    tvs_config cfg{};
    GridDev gd{};
    tvs::MlpCfg mlp{};
    hipStream_t stream = nullptr;
    int64_t nvox = 0;               // words of a device image (tiled layout, padding included)
    int64_t nimg = 0;               // voxels of an image at the ABI (nx * ny * nz)
    int64_t ntiles = 0;
    uint64_t budget = 0;
    uint64_t bytes = 0;
    std::string err;

    // image side (float64, tiled layout)
    double *x = nullptr, *g = nullptr;
    double *x0 = nullptr;           // initial iterate, the starting image of batches
    float *xio = nullptr;           // float32 staging of the image at the ABI
    double *part = nullptr, *scal = nullptr;
    uint32_t *ticket = nullptr;
    int64_t nparts = 0;
    uint32_t *flags = nullptr;      // kNumFlags device flags
    long long *dot = nullptr;       // 3 x B fixed-point row dot products

    // histories and the tile lists of their DROP blocks
    bool loaded = false;
    int64_t nh = 0;
    float *hist = nullptr;          // 13 * nh floats
    int64_t *row_off = nullptr;     // nh + 1, entry offsets in walk order
    float *norm2 = nullptr;         // nh
    double *s1i = nullptr;          // entry-side MLP table (3 per vertex depth)
    int64_t nj = 0;
    int64_t *seg_off = nullptr;     // nh + 1
    int32_t *order = nullptr;       // nh: each chunk's histories by decreasing row length
    uint64_t *segtab = nullptr;     // nseg: global entry index of each segment's first entry
    int64_t nseg = 0;
    int64_t *bt_off = nullptr;      // nblocks * nact + 1 list starts, slots in order per block
    int32_t *act = nullptr;         // tiles that some block's lists cross (slot -> tile)
    int32_t *slot_of = nullptr;     // ntiles: tile -> slot, -1 for a tile no list crosses
    int64_t nact = 0;
    int64_t nblocks = 0;
    // entries: the store, or a ring of chunk buffers on the fly
    uint32_t *meta[kChunkBuffers] = {};
    float *ch32[kChunkBuffers] = {};
    __half *ch16 = nullptr;
    uint16_t *chq = nullptr;        // fixed-point store: low 16 bits of the chord codes
    float chord_max = 0.0f;         // longest chord of the loaded rows (float32, rounded up)
    double qunit = 0.0;             // fixed-point store: mm per code unit
    double qinv = 0.0;              // 1 / qunit
    uint32_t qmax = 0;              // largest code (2^bits - 1)
    uint32_t qshift = 31;           // tag bit that holds the code's bit 16
    uint32_t rowmask = 0xffffffu;   // row field of the tags
    int64_t cap = 0;                // entries per buffer
    int nbuf = 0;
    int64_t cbase = 0;              // ring position of the next sweep's first chunk
    hipStream_t fill_stream = nullptr;          // row formation of the next chunks
    hipEvent_t ev_filled[kChunkBuffers] = {};
    hipEvent_t ev_free[kChunkBuffers] = {};
    int64_t nnz = 0, max_row = 0, skipped = 0;
    int64_t chunk = 0;              // histories per chunk (a multiple of B)
    std::vector<int64_t> chunk_base;  // entry offset of each chunk start (and the end)
    double big = 0.0, dot_max = 0.0;  // fixed-point ranges of the DROP kernels
    int threads = 256;              // threads per tile workgroup
    int split = 0;                  // 1: two launches per block
    int bthreads = 256;             // batched DROP step: threads per workgroup
    int bgroup = 4;                 // batched DROP step: settings per pass through LDS
    int64_t fill_wgs = 0;           // grid cap of the sweep's row formation (0: none)
    int fill_wide_pct = 0;          // chunks formed at the row kernel's full occupancy, %

    // cycle state
    int64_t k = 0, ell = 0;
    uint64_t rng = 0;
    bool seeded = false;
    std::vector<tvs_step_log> log;
    int64_t tries = 0;
    // checked cycles keep ell and the RNG state on the device (sched) and
    // write their step records there (dlog); dev_sched: the device copy is
    // the current one, to be copied back (after ev_sched) before the host
    // uses ell again or reports the log
    tvs::SchedDev *sched = nullptr;
    tvs_step_log *dlog = nullptr;
    int64_t dlog_n = 0;
    bool dev_sched = false;
    hipEvent_t ev_sched = nullptr;
    double *cpart = nullptr;        // partial sums of the device-side check

    // timing: HIP events recorded on the launch stream around every phase of
    // the last tvs_iterate call, resolved lazily by tvs_get_stats
    std::vector<hipEvent_t> tev;
    size_t tev_used = 0;
    // kind: 0 TV steps, 1 sweep, 2 rows, 3 DROP, 4 first / 5 second launch of a sampled block
    struct Span { int kind; size_t a, b; };
    std::vector<Span> spans;
    bool timed = false;
    double last_sweep_ms = 0, last_tv_ms = 0, last_rows_ms = 0;
    double tot_ms[6] = {0, 0, 0, 0, 0, 0};
    int64_t tot_n[6] = {0, 0, 0, 0, 0, 0};

    // batched reconstructions
    struct Batch {
        int S = 0;
        bool valid = false;
        std::vector<tvs_params> p;
        tvs::BatchBuffers b;
        long long *dot = nullptr;   // 3 x B x S
        int64_t k = 0;
        std::vector<int64_t> ell;
        std::vector<uint64_t> rng;
        int64_t beta_cap = 0;
        double ms_total = 0;
        int64_t cycles = 0;
    } batch;
    // fork/join events of the captured batched cycle (the fill stream's row
    // formation beside the batched chain); only ever recorded in capture
    hipEvent_t bev_fork = nullptr;
    hipEvent_t bev_filled[kChunkBuffers] = {};
    hipEvent_t bev_free[kChunkBuffers] = {};
};

namespace {

int fail(tvs_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(ctx, TVS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
int dalloc(tvs_ctx *ctx, T **p, size_t count)
{
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);
    if (ctx->bytes + bytes > ctx->budget)
        return fail(ctx, TVS_ENOMEM,
                    "footprint " + std::to_string(ctx->bytes + bytes) + " B exceeds budget " +
                        std::to_string(ctx->budget) + " B");
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, TVS_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    *p = static_cast<T *>(q);
    ctx->bytes += bytes;
    return TVS_OK;
}

template <typename T>
void dfree(tvs_ctx *ctx, T **p, size_t count)
{
    if (*p) {
        (void)hipFree(*p);
        size_t bytes = count * sizeof(T);
        if (bytes == 0) bytes = sizeof(T);
        ctx->bytes -= std::min<uint64_t>(ctx->bytes, bytes);
        *p = nullptr;
    }
}

int64_t bt_len(const tvs_ctx *ctx) { return ctx->nblocks * ctx->nact + 1; }

// Ring buffer of chunk c of the current sweep (on the fly).
int chunk_buffer(const tvs_ctx *ctx, int64_t c) { return (int)((ctx->cbase + c) % ctx->nbuf); }

void free_histories(tvs_ctx *ctx)
{
    dfree(ctx, &ctx->hist, (size_t)(kNumStreams * ctx->nh));
    dfree(ctx, &ctx->row_off, (size_t)(ctx->nh + 1));
    dfree(ctx, &ctx->norm2, (size_t)ctx->nh);
    dfree(ctx, &ctx->seg_off, (size_t)(ctx->nh + 1));
    dfree(ctx, &ctx->order, (size_t)ctx->nh);
    dfree(ctx, &ctx->s1i, (size_t)(3 * ctx->nj));
    ctx->nj = 0;
    ctx->mlp.s1i = nullptr;
    ctx->mlp.nj = 0;
    dfree(ctx, &ctx->segtab, (size_t)ctx->nseg);
    dfree(ctx, &ctx->bt_off, (size_t)bt_len(ctx));
    dfree(ctx, &ctx->act, (size_t)std::max<int64_t>(ctx->nact, 1));
    dfree(ctx, &ctx->slot_of, (size_t)std::max<int64_t>(ctx->ntiles, 1));
    ctx->nact = 0;
    for (int q = 0; q < kChunkBuffers; q++) {
        dfree(ctx, &ctx->meta[q], (size_t)ctx->cap);
        dfree(ctx, &ctx->ch32[q], (size_t)ctx->cap);
    }
    dfree(ctx, &ctx->ch16, (size_t)ctx->cap);
    dfree(ctx, &ctx->chq, (size_t)ctx->cap);
    ctx->chord_max = 0.0f;
    ctx->qunit = ctx->qinv = 0.0;
    ctx->qmax = 0;
    ctx->qshift = 31;
    ctx->rowmask = 0xffffffu;
    ctx->loaded = false;
    ctx->nh = 0;
    ctx->nseg = 0;
    ctx->nblocks = 0;
    ctx->cap = 0;
    ctx->nbuf = 0;
    ctx->cbase = 0;
    ctx->nnz = ctx->max_row = ctx->skipped = 0;
    ctx->chunk_base.clear();
}

void free_batch(tvs_ctx *ctx)
{
    auto &B = ctx->batch;
    const size_t n = (size_t)(ctx->nvox * B.S);
    dfree(ctx, &B.b.x, n);
    dfree(ctx, &B.b.g, n);
    dfree(ctx, &B.b.part, (size_t)(tvs::batch_num_parts(ctx->gd, std::max(B.S, 1)) * B.S));
    dfree(ctx, &B.b.ticket, (size_t)4);
    dfree(ctx, &B.b.norm2, (size_t)B.S);
    dfree(ctx, &B.b.lambda, (size_t)B.S);
    dfree(ctx, &B.b.eps, (size_t)B.S);
    dfree(ctx, &B.b.beta_tab, (size_t)B.beta_cap);
    dfree(ctx, &B.b.cyc, (size_t)4);
    dfree(ctx, &B.dot, (size_t)(3 * (int64_t)ctx->cfg.block_size * B.S));
    B = tvs_ctx::Batch();
}

HistDev hist_dev(const tvs_ctx *ctx)
{
    return HistDev{ctx->hist, ctx->nh};
}

tvs::TvBuffers tv_bufs(tvs_ctx *ctx)
{
    return tvs::TvBuffers{ctx->g, ctx->part, ctx->ticket, ctx->scal, ctx->nparts};
}

hipStream_t pick(tvs_ctx *ctx, void *stream)
{
    return stream ? static_cast<hipStream_t>(stream) : ctx->stream;
}

void reset_state(tvs_ctx *ctx)
{
    ctx->k = 0;
    ctx->ell = 0;
    ctx->rng = 0;
    ctx->seeded = false;
    ctx->log.clear();
    ctx->tries = 0;
    ctx->dev_sched = false;
    ctx->dlog_n = 0;
}

// Copies the schedule and step records of checked cycles back from the
// device (waits for the work of the last checked call).
int settle_sched(tvs_ctx *ctx)
{
    if (!ctx->dev_sched) return TVS_OK;
    HIPCHK(hipEventSynchronize(ctx->ev_sched));
    tvs::SchedDev sd{};
    HIPCHK(hipMemcpy(&sd, ctx->sched, sizeof(sd), hipMemcpyDeviceToHost));
    std::vector<tvs_step_log> recs((size_t)ctx->dlog_n);
    if (ctx->dlog_n > 0)
        HIPCHK(hipMemcpy(recs.data(), ctx->dlog, sizeof(tvs_step_log) * (size_t)ctx->dlog_n,
                         hipMemcpyDeviceToHost));
    for (const auto &r : recs) {
        ctx->log.push_back(r);
        ctx->tries += r.tries;
    }
    ctx->ell = sd.ell;
    ctx->rng = sd.rng;
    ctx->dlog_n = 0;
    ctx->dev_sched = false;
    return TVS_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Records a timing event on st; returns its index in the pool (or -1). Pool
// events skip the system-scope fence: they carry timestamps only, and the fence
// (an L2 write-back) would otherwise be timed with the work it brackets.
long mark(tvs_ctx *ctx, hipStream_t st)
{
    if (ctx->tev_used == ctx->tev.size()) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return -1;
        ctx->tev.push_back(e);
    }
    if (hipEventRecord(ctx->tev[ctx->tev_used], st) != hipSuccess) return -1;
    return (long)ctx->tev_used++;
}

// Reserves an event of the pool without recording it (recorded by a launch).
long slot(tvs_ctx *ctx)
{
    if (ctx->tev_used == ctx->tev.size()) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return -1;
        ctx->tev.push_back(e);
    }
    return (long)ctx->tev_used++;
}

void span(tvs_ctx *ctx, int kind, long a, long b)
{
    if (a >= 0 && b >= 0) ctx->spans.push_back({kind, (size_t)a, (size_t)b});
}

// Pool events for the kernels of one sampled block, stamped by the launches
// themselves: the first launch (kind 4) and, when the step is split in two
// launches, the second (kind 5).
bool ktimer(tvs_ctx *ctx, tvs::KTimer &kt, bool two)
{
    const int n = two ? 4 : 2;
    long q[4] = {-1, -1, -1, -1};
    for (int i = 0; i < n; i++)
        if ((q[i] = slot(ctx)) < 0) return false;
    for (int i = 0; i < n; i++) kt.e[i] = ctx->tev[(size_t)q[i]];
    span(ctx, 4, q[0], q[1]);
    if (two) span(ctx, 5, q[2], q[3]);
    return true;
}

// Checks the device flags raised by the DROP and row kernels (waits for the
// work queued on st).
int check_flags(tvs_ctx *ctx, hipStream_t st)
{
    uint32_t f[kNumFlags] = {};
    HIPCHK(hipMemcpyAsync(f, ctx->flags, sizeof(f), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (f[kFlagLists] || (f[kFlagRange] & 2u))
        return fail(ctx, TVS_EDEVICE, "a row walk disagreed with its load-time tile lists");
    if (f[kFlagRange])
        return fail(ctx, TVS_ERANGE,
                    "a DROP product |a_ij x_j| left the fixed-point range (image values too "
                    "large); set a new image to clear");
    return TVS_OK;
}

// One block's tile lists as the DROP kernels see them.
TileBlock block_view(tvs_ctx *ctx, int64_t b, long long *dot_base, int64_t dot_stride)
{
    const int64_t B = ctx->cfg.block_size;
    const bool otf = ctx->cfg.path_mode == TVS_PATH_ON_THE_FLY;
    const int64_t c = otf ? (b * B) / ctx->chunk : 0;
    const int buf = otf ? chunk_buffer(ctx, c) : 0;
    TileBlock t;
    t.meta = ctx->meta[buf];
    t.ch32 = ctx->ch32[buf];
    t.ch16 = ctx->ch16;
    t.chq = ctx->chq;
    t.qunit = ctx->qunit;
    t.qshift = ctx->qshift;
    t.rowmask = ctx->rowmask;
    t.toff = ctx->bt_off + b * ctx->nact;
    t.base = otf ? ctx->chunk_base[(size_t)c] : 0;
    t.wepl = ctx->hist + 12 * ctx->nh + b * B;
    t.n2 = ctx->norm2 + b * B;
    t.dot = dot_base + (b % 3) * dot_stride;
    t.rows = (uint32_t)std::min<int64_t>(B, ctx->nh - b * B);
    t.valid = 1;
    return t;
}

// Forms the rows of chunk c (histories [c*chunk, c*chunk + n)) into its buffer.
tvs::TileFill chunk_fill(tvs_ctx *ctx, int64_t c, int64_t n)
{
    tvs::TileFill f;
    f.first = c * ctx->chunk;
    f.n = n;
    f.B = ctx->cfg.block_size;
    f.seg_off = ctx->seg_off;
    f.segdst = reinterpret_cast<const int64_t *>(ctx->segtab);
    f.base = ctx->chunk_base[(size_t)c];
    f.meta = ctx->meta[chunk_buffer(ctx, c)];
    f.ch32 = ctx->ch32[chunk_buffer(ctx, c)];
    f.ch16 = ctx->ch16;
    f.cap = ctx->cap;
    f.norm2 = ctx->norm2;
    f.err = ctx->flags + kFlagLists;
    f.max_wgs = ctx->fill_wgs;
    f.order = ctx->order;
    // beside the DROP chain: chunk c at full occupancy when the running count
    // of such chunks steps up at c (fill_wide_pct of them, spread evenly),
    // else held at two waves per SIMD
    const int64_t pct = ctx->fill_wide_pct;
    f.room = ((c + 1) * pct / 100 > c * pct / 100) ? 0 : 1;
    return f;
}

// One P_T sweep over the loaded histories (the first `limit` of them when
// limit >= 0, a multiple of B: used to time launch shapes).
int run_sweep(tvs_ctx *ctx, double lambda, hipStream_t st, int64_t limit = -1)
{
    const int64_t B = ctx->cfg.block_size;
    const int64_t nh_run = (limit >= 0) ? std::min(limit, ctx->nh) : ctx->nh;
    if (nh_run <= 0) return TVS_OK;
    const int64_t nb = (nh_run + B - 1) / B;
    const bool otf = ctx->cfg.path_mode == TVS_PATH_ON_THE_FLY;
    const int64_t step = otf ? ctx->chunk : ctx->nh;
    const int64_t nchunks = (nh_run + step - 1) / step;
    hipStream_t fs = ctx->fill_stream;
    HIPCHK(tvs::launch_zero_i64(ctx->dot, 3 * B, st));
    // a chunk is always formed whole, also when the sweep stops inside it:
    // its rows are formed in length order, so the first n of them are not
    // the histories of the first blocks
    auto fill = [&](int64_t c) -> int {
        const int64_t n = std::min(step, ctx->nh - c * step);
        tvs::TileFill f = chunk_fill(ctx, c, n);
        HIPCHK(hipStreamWaitEvent(fs, ctx->ev_free[chunk_buffer(ctx, c)], 0));
        long a = mark(ctx, fs);
        HIPCHK(tvs::launch_rows_fill_tiled(ctx->gd, hist_dev(ctx), ctx->mlp, f, fs));
        span(ctx, 2, a, mark(ctx, fs));
        HIPCHK(hipEventRecord(ctx->ev_filled[chunk_buffer(ctx, c)], fs));
        return TVS_OK;
    };
    const int64_t NB = ctx->nbuf;
    if (otf) {
        for (int64_t c = 0; c < std::min<int64_t>(NB, nchunks); c++) {
            int rc = fill(c);
            if (rc) return rc;
        }
    }
    long e0 = mark(ctx, st);
    for (int64_t b = 0; b <= nb; b++) {
        const bool has_c = b < nb;
        const int64_t c = has_c ? (b * B) / step : -1;
        const bool first_of_chunk = has_c && (b * B) % step == 0;
        if (otf && first_of_chunk)
            HIPCHK(hipStreamWaitEvent(st, ctx->ev_filled[chunk_buffer(ctx, c)], 0));
        tvs::DropTileArgs A;
        if (b > 0) A.P = block_view(ctx, b - 1, ctx->dot, B);
        if (has_c) A.C = block_view(ctx, b, ctx->dot, B);
        A.x = ctx->x;
        A.lambda = lambda;
        A.big = ctx->big;
        A.dot_max = ctx->dot_max;
        A.zero = ctx->dot + ((b + 1) % 3) * B;
        A.B = B;
        A.err = ctx->flags + kFlagRange;
        A.tiles = ctx->act;
        A.nact = ctx->nact;
        const bool samp = ctx->cfg.time_sample > 0 && has_c && b > 0 &&
                          b % ctx->cfg.time_sample == 0;
        tvs::KTimer kt;
        const bool timed = samp && ktimer(ctx, kt, ctx->split != 0);
        HIPCHK(tvs::launch_drop_tiles(A, ctx->ntiles, ctx->threads, ctx->split, st,
                                      timed ? &kt : nullptr));
        if (otf && first_of_chunk && c >= 1) {
            // the launch above was the last to read chunk c - 1's buffer,
            // which takes chunk c - 1 + NB next
            HIPCHK(hipEventRecord(ctx->ev_free[chunk_buffer(ctx, c - 1)], st));
            if (c - 1 + NB < nchunks) {
                int rc = fill(c - 1 + NB);
                if (rc) return rc;
            }
        }
    }
    span(ctx, 3, e0, mark(ctx, st));
    if (otf) {
        HIPCHK(hipEventRecord(ctx->ev_free[chunk_buffer(ctx, nchunks - 1)], st));
        // the ring continues with the next sweep, whose first chunks take the
        // buffers freed first
        ctx->cbase = (ctx->cbase + nchunks) % NB;
    }
    return TVS_OK;
}

int validate_params(tvs_ctx *ctx, const tvs_params *p)
{
    if (!p) return fail(ctx, TVS_EINVAL, "params is NULL");
    if (!finite_pos(p->lambda)) return fail(ctx, TVS_EINVAL, "lambda must be finite and > 0");
    if (p->variant < 0 || p->variant > 2) return fail(ctx, TVS_EINVAL, "unknown variant");
    if (p->variant != TVS_OTVS && !(p->alpha > 0.0 && p->alpha < 1.0))
        return fail(ctx, TVS_EINVAL, "alpha must lie in (0, 1)");
    if (p->N < 0) return fail(ctx, TVS_EINVAL, "N must be >= 0");
    if (!(p->tv_eps >= 0.0) || !std::isfinite(p->tv_eps))
        return fail(ctx, TVS_EINVAL, "tv_eps must be finite and >= 0");
    if (p->variant == TVS_DECOUPLED && !(p->gamma > 0.0 && p->gamma < 1.0))
        return fail(ctx, TVS_EINVAL, "gamma must lie in (0, 1)");
    return TVS_OK;
}

// Row lengths of histories [first, first + n) into row_off_dev (n + 1).
int count_rows(tvs_ctx *ctx, int64_t first, int64_t n, int64_t *row_off_dev, hipStream_t st)
{
    int32_t *cnt = nullptr;
    int64_t *tmp = nullptr;
    int rc = dalloc(ctx, &cnt, (size_t)std::max<int64_t>(n, 1));
    if (rc) return rc;
    rc = dalloc(ctx, &tmp, (size_t)tvs::scan_tmp_elems(n) + 1);
    if (rc) {
        dfree(ctx, &cnt, (size_t)std::max<int64_t>(n, 1));
        return rc;
    }
    hipError_t e =
        tvs::launch_rows_count(ctx->gd, hist_dev(ctx), ctx->mlp, first, n, cnt, nullptr, st);
    if (e == hipSuccess) e = tvs::launch_scan(cnt, n, row_off_dev, tmp, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree(ctx, &cnt, (size_t)std::max<int64_t>(n, 1));
    dfree(ctx, &tmp, (size_t)tvs::scan_tmp_elems(n) + 1);
    if (e != hipSuccess) return fail(ctx, TVS_EDEVICE, std::string("row count: ") + hipGetErrorString(e));
    return TVS_OK;
}

// The tiles that some block's lists cross (a tile outside the scanned
// object has no entry in any block), from the (block, tile) list lengths:
// the DROP steps launch one workgroup per such tile only, in order of
// decreasing entries over the scan, so that the longest lists are
// dispatched first and do not trail the step.  Workgroup i of a step takes
// slot i: tile act[i], whose lists are laid out in slot order (slot_of
// inverts act; -1 for a tile no list crosses).  At least one tile is kept,
// so that a step always has a workgroup to clear the next dot-product
// buffer.
int build_active_tiles(tvs_ctx *ctx, const uint32_t *btc, hipStream_t st)
{
    const int64_t nt = ctx->ntiles;
    uint32_t *total = nullptr;
    int rc = dalloc(ctx, &total, (size_t)std::max<int64_t>(nt, 1));
    if (rc) return rc;
    std::vector<uint32_t> f((size_t)std::max<int64_t>(nt, 1), 0u);
    hipError_t e = tvs::launch_tile_totals(btc, ctx->nblocks, nt, total, st);
    if (e == hipSuccess && nt > 0)
        e = hipMemcpyAsync(f.data(), total, sizeof(uint32_t) * nt, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree(ctx, &total, (size_t)std::max<int64_t>(nt, 1));
    if (e != hipSuccess) return fail(ctx, TVS_EDEVICE, std::string("active tiles: ") + hipGetErrorString(e));
    std::vector<int32_t> a;
    for (int64_t T = 0; T < nt; T++)
        if (f[(size_t)T]) a.push_back((int32_t)T);
    std::stable_sort(a.begin(), a.end(),
                     [&](int32_t x, int32_t y) { return f[(size_t)x] > f[(size_t)y]; });
    if (a.empty()) a.push_back(0);
    std::vector<int32_t> inv((size_t)std::max<int64_t>(nt, 1), -1);
    for (size_t i = 0; i < a.size(); i++) inv[(size_t)a[i]] = (int32_t)i;
    rc = dalloc(ctx, &ctx->act, a.size());
    if (!rc) rc = dalloc(ctx, &ctx->slot_of, inv.size());
    if (rc) return rc;
    ctx->nact = (int64_t)a.size();
    e = hipMemcpyAsync(ctx->act, a.data(), sizeof(int32_t) * a.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->slot_of, inv.data(), sizeof(int32_t) * inv.size(),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(ctx, TVS_EDEVICE, std::string("active tiles: ") + hipGetErrorString(e));
    return TVS_OK;
}

// Lays out the tile lists of every block: row and segment counts, each
// segment's place in its (block, tile) list, the list starts.  Sets nnz,
// max_row, skipped, nseg, nblocks and the chunking.
int build_tile_lists(tvs_ctx *ctx, hipStream_t st)
{
    const int64_t n = ctx->nh, B = ctx->cfg.block_size;
    const int64_t nbt = ((n + B - 1) / B) * ctx->ntiles;
    int32_t *cnt = nullptr, *cseg = nullptr;
    uint32_t *btc = nullptr, *sbc = nullptr;   // list lengths by (block, tile), by (block, slot)
    int64_t nsbc = 0;
    int64_t *tmp = nullptr;
    // scan scratch, later also the gathered block starts
    const int64_t ntmp = std::max(tvs::scan_tmp_elems(std::max(n, nbt)) + 1, (n + B - 1) / B + 1);
    auto cleanup = [&]() {
        dfree(ctx, &cnt, (size_t)std::max<int64_t>(n, 1));
        dfree(ctx, &cseg, (size_t)std::max<int64_t>(n, 1));
        dfree(ctx, &btc, (size_t)std::max<int64_t>(nbt, 1));
        dfree(ctx, &sbc, (size_t)std::max<int64_t>(nsbc, 1));
        dfree(ctx, &tmp, (size_t)ntmp);
    };
    int rc = dalloc(ctx, &cnt, (size_t)std::max<int64_t>(n, 1));
    if (!rc) rc = dalloc(ctx, &cseg, (size_t)std::max<int64_t>(n, 1));
    if (!rc) rc = dalloc(ctx, &tmp, (size_t)ntmp);
    if (rc) {
        cleanup();
        return rc;
    }
    HistDev hd = hist_dev(ctx);
    hipError_t e = tvs::launch_rows_count(ctx->gd, hd, ctx->mlp, 0, n, cnt, cseg, st);
    if (e == hipSuccess) e = tvs::launch_scan(cnt, n, ctx->row_off, tmp, st);
    if (e == hipSuccess) e = tvs::launch_scan(cseg, n, ctx->seg_off, tmp, st);
    std::vector<int64_t> off((size_t)n + 1);
    int64_t nseg = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(off.data(), ctx->row_off, sizeof(int64_t) * (n + 1),
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&nseg, ctx->seg_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        cleanup();
        return fail(ctx, TVS_EDEVICE, std::string("row count: ") + hipGetErrorString(e));
    }
    dfree(ctx, &cnt, (size_t)std::max<int64_t>(n, 1));
    dfree(ctx, &cseg, (size_t)std::max<int64_t>(n, 1));
    const int64_t total = off[(size_t)n];
    int64_t mx = 0, sk = 0;
    for (int64_t i = 0; i < n; i++) {
        const int64_t len = off[(size_t)i + 1] - off[(size_t)i];
        mx = std::max(mx, len);
        sk += (len == 0);
    }
    ctx->nnz = total;
    ctx->max_row = mx;
    ctx->skipped = sk;
    ctx->nseg = nseg;
    ctx->nblocks = (n + B - 1) / B;
    int64_t chunk = ctx->cfg.chunk_histories;
    if (chunk <= 0) {
        // about 2^20 histories, as even as whole blocks allow: the row
        // formation of the next sweep's first chunk waits for the DROP chain
        // to leave that chunk's buffer, i.e. to finish the next-to-last chunk,
        // so a small last chunk would leave the formation stream idle
        const int64_t target = std::max<int64_t>(B, ((int64_t)1 << 20) / B * B);
        const int64_t parts = std::max<int64_t>(1, (n + target - 1) / target);
        chunk = ((n + parts - 1) / parts + B - 1) / B * B;
        chunk = std::max<int64_t>(chunk, B);
    } else {
        chunk = (chunk + B - 1) / B * B;
    }
    ctx->chunk = std::max<int64_t>(chunk, 1);
    for (int64_t f = 0; f < n; f += ctx->chunk) ctx->chunk_base.push_back(off[(size_t)f]);
    ctx->chunk_base.push_back(total);
    // processing order of the row passes: within each DROP block, histories
    // by decreasing row length (a counting sort), so that the lanes of a
    // wavefront walk rows of similar length while a block's tile lists are
    // still written together (their partly written lines meet in the L2
    // before they are evicted); blocks never straddle a chunk.  Each
    // segment's place is fixed below, so the order changes no result
    {
        std::vector<int32_t> ord((size_t)n);
        std::vector<int64_t> cnt_len((size_t)mx + 2);
        for (int64_t f0 = 0; f0 < n; f0 += B) {
            const int64_t f1 = std::min(n, f0 + B);
            std::fill(cnt_len.begin(), cnt_len.end(), 0);
            for (int64_t i = f0; i < f1; i++) cnt_len[(size_t)(mx - (off[(size_t)i + 1] - off[(size_t)i]))]++;
            int64_t pos = f0;
            for (size_t q = 0; q < cnt_len.size(); q++) {
                const int64_t c0 = cnt_len[q];
                cnt_len[q] = pos;
                pos += c0;
            }
            for (int64_t i = f0; i < f1; i++)
                ord[(size_t)cnt_len[(size_t)(mx - (off[(size_t)i + 1] - off[(size_t)i]))]++] = (int32_t)i;
        }
        rc = dalloc(ctx, &ctx->order, (size_t)n);
        if (rc) {
            cleanup();
            return rc;
        }
        e = hipMemcpyAsync(ctx->order, ord.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            cleanup();
            return fail(ctx, TVS_EDEVICE, std::string("row order: ") + hipGetErrorString(e));
        }
    }
    // integer ranges of the DROP sums: no voxel takes more than 2B entries of
    // one block, no row more than max_row entries
    ctx->big = 2097152.0 / (double)B;                              // 2^21 / B
    ctx->dot_max = 67108864.0 / (double)std::max<int64_t>(mx, 1);  // 2^26 / max_row

    rc = dalloc(ctx, &ctx->segtab, (size_t)nseg);
    if (!rc) rc = dalloc(ctx, &btc, (size_t)std::max<int64_t>(nbt, 1));
    if (rc) {
        cleanup();
        return rc;
    }
    e = hipMemsetAsync(btc, 0, sizeof(uint32_t) * std::max<int64_t>(nbt, 1), st);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->flags, 0, sizeof(uint32_t) * kNumFlags, st);
    if (e == hipSuccess)
        e = tvs::launch_rows_seg(ctx->gd, hd, ctx->mlp, n, B, ctx->seg_off, btc, ctx->segtab,
                                 ctx->flags + kFlagLists, ctx->flags + kFlagChordMax, ctx->order,
                                 st);
    if (e != hipSuccess) {
        cleanup();
        return fail(ctx, TVS_EDEVICE, std::string("tile lists: ") + hipGetErrorString(e));
    }
    // the dispatch slots, then the lists of every block laid out in slot
    // order: a step's workgroup i finds its list bounds at [b * nact + i]
    // without first looking up its tile
    rc = build_active_tiles(ctx, btc, st);
    nsbc = ctx->nblocks * ctx->nact;
    if (!rc) rc = dalloc(ctx, &ctx->bt_off, (size_t)bt_len(ctx));
    if (!rc) rc = dalloc(ctx, &sbc, (size_t)std::max<int64_t>(nsbc, 1));
    if (rc) {
        cleanup();
        return rc;
    }
    e = tvs::launch_slot_counts(btc, ctx->act, ctx->nact, ctx->nblocks, ctx->ntiles, sbc, st);
    if (e == hipSuccess)
        e = tvs::launch_scan(reinterpret_cast<const int32_t *>(sbc), nsbc, ctx->bt_off, tmp, st);
    if (e == hipSuccess)
        e = tvs::launch_seg_dest(ctx->gd, n, B, ctx->seg_off, ctx->bt_off, ctx->slot_of,
                                 ctx->nact, ctx->segtab, ctx->flags + kFlagLists, st);
    // every block's lists must add up to the block's entries (the block
    // starts are gathered into the freed count buffer, then copied)
    std::vector<int64_t> starts((size_t)ctx->nblocks + 1);
    if (e == hipSuccess && ctx->nblocks > 0)
        e = tvs::launch_pick(ctx->bt_off, ctx->nact, ctx->nblocks + 1, tmp, st);
    if (e == hipSuccess && ctx->nblocks > 0)
        e = hipMemcpyAsync(starts.data(), tmp, sizeof(int64_t) * (ctx->nblocks + 1),
                           hipMemcpyDeviceToHost, st);
    uint32_t fl[kNumFlags] = {};
    if (e == hipSuccess)
        e = hipMemcpyAsync(fl, ctx->flags, sizeof(fl), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    cleanup();
    if (e != hipSuccess) return fail(ctx, TVS_EDEVICE, std::string("tile lists: ") + hipGetErrorString(e));
    if (fl[kFlagLists])
        return fail(ctx, TVS_EDEVICE, "tile lists: a row walk disagreed with the count pass");
    std::memcpy(&ctx->chord_max, &fl[kFlagChordMax], sizeof(float));
    for (int64_t b = 0; b <= ctx->nblocks && ctx->nblocks > 0; b++) {
        const int64_t want = (b < ctx->nblocks) ? off[(size_t)(b * B)] : total;
        if (starts[(size_t)b] != want)
            return fail(ctx, TVS_EDEVICE,
                        "tile lists disagree with the row lengths at block " + std::to_string(b) +
                            " of " + std::to_string(ctx->nblocks) + ": " +
                            std::to_string(starts[(size_t)b]) + " != " + std::to_string(want));
    }
    return TVS_OK;
}

// Allocates the entry buffers and, for a path store, forms every row now.
int form_entries(tvs_ctx *ctx, hipStream_t st)
{
    const bool otf = ctx->cfg.path_mode == TVS_PATH_ON_THE_FLY;
    int64_t cap = ctx->nnz;
    if (otf) {
        cap = 0;
        for (size_t q = 0; q + 1 < ctx->chunk_base.size(); q++)
            cap = std::max(cap, ctx->chunk_base[q + 1] - ctx->chunk_base[q]);
    }
    ctx->cap = std::max<int64_t>(cap, 1);
    const int64_t nchunks = (int64_t)ctx->chunk_base.size() - 1;
    ctx->nbuf = otf ? (int)std::max<int64_t>(1, std::min<int64_t>(kChunkBuffers, nchunks)) : 1;
    ctx->cbase = 0;
    int rc = TVS_OK;
    for (int q = 0; q < ctx->nbuf && !rc; q++) {
        rc = dalloc(ctx, &ctx->meta[q], (size_t)ctx->cap);
        if (!rc) {
            if (ctx->cfg.path_mode == TVS_PATH_STORE_F16) rc = dalloc(ctx, &ctx->ch16, (size_t)ctx->cap);
            else if (ctx->cfg.path_mode == TVS_PATH_STORE_Q16) rc = dalloc(ctx, &ctx->chq, (size_t)ctx->cap);
            else rc = dalloc(ctx, &ctx->ch32[q], (size_t)ctx->cap);
        }
        // entries start as (row 0, word 0, chord 0): never an index out of range
        if (!rc) HIPCHK(hipMemsetAsync(ctx->meta[q], 0, sizeof(uint32_t) * ctx->cap, st));
        if (!rc && ctx->ch32[q]) HIPCHK(hipMemsetAsync(ctx->ch32[q], 0, sizeof(float) * ctx->cap, st));
    }
    if (!rc && ctx->ch16) HIPCHK(hipMemsetAsync(ctx->ch16, 0, sizeof(__half) * ctx->cap, st));
    if (!rc && ctx->chq) HIPCHK(hipMemsetAsync(ctx->chq, 0, sizeof(uint16_t) * ctx->cap, st));
    if (rc) return rc;
    if (ctx->chq) {
        // fixed-point chords: rb bits of a tag hold the row within its block
        // (B rows), the 24 - rb above them the code's high bits, so a code
        // has 16 + 24 - rb bits (at most 30); the unit is the longest chord /
        // the largest code, made a little larger so that the longest chord's
        // code stays in range after rounding
        const uint32_t B = (uint32_t)ctx->cfg.block_size;
        uint32_t rb = 0;
        while (rb < 24 && ((uint32_t)1 << rb) < B) rb++;
        const uint32_t bits = std::min<uint32_t>(30, 16 + (24 - rb));
        ctx->rowmask = rb ? (((uint32_t)1 << rb) - 1u) : 0u;
        ctx->qshift = kTileShiftHost + rb;
        ctx->qmax = (uint32_t)(((uint64_t)1 << bits) - 1u);
        const double m = ctx->chord_max > 0.0f ? (double)ctx->chord_max : 1.0;
        ctx->qunit = m * (1.0 + 1.0 / 1048576.0) / (double)ctx->qmax;
        ctx->qinv = 1.0 / ctx->qunit;
    }
    if (otf) {
        // the first sweep's row formation runs on the fill stream: it must
        // not start before these clears, or they overwrite formed entries
        for (int q = 0; q < kChunkBuffers; q++) HIPCHK(hipEventRecord(ctx->ev_free[q], st));
        return TVS_OK;
    }
    if (ctx->nh == 0) return TVS_OK;
    tvs::TileFill f;
    f.first = 0;
    f.n = ctx->nh;
    f.B = ctx->cfg.block_size;
    f.seg_off = ctx->seg_off;
    f.segdst = reinterpret_cast<const int64_t *>(ctx->segtab);
    f.base = 0;
    f.meta = ctx->meta[0];
    f.ch32 = ctx->ch32[0];
    f.ch16 = ctx->ch16;
    f.chq = ctx->chq;
    f.qinv = ctx->qinv;
    f.qmax = ctx->qmax;
    f.qshift = ctx->qshift;
    f.cap = ctx->cap;
    f.norm2 = ctx->norm2;
    f.err = ctx->flags + kFlagLists;
    f.order = ctx->order;
    hipError_t e = tvs::launch_rows_fill_tiled(ctx->gd, hist_dev(ctx), ctx->mlp, f, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(ctx, TVS_EDEVICE, std::string("row fill: ") + hipGetErrorString(e));
    return check_flags(ctx, st);
}

}  // namespace

extern "C" {

void tvs_config_default(tvs_config *cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->block_size = 3200;
    cfg->path_mode = TVS_PATH_ON_THE_FLY;
    cfg->mlp_step_mm = 0.0;
    cfg->mlp_log_term = 1;
    cfg->mlp_const_power = 0;
    cfg->chunk_histories = 0;
    cfg->hbm_budget_bytes = 0;
    cfg->device = 0;
    cfg->max_tries = 0;
    cfg->sweep_kernel = 0;
    cfg->tile_threads = 0;
    cfg->time_sample = 0;
    cfg->fill_wgs_per_cu = 0;
    cfg->fill_wide_pct = -1;
}

const char *tvs_strerror(int status)
{
    switch (status) {
    case TVS_OK: return "ok";
    case TVS_EINVAL: return "invalid argument";
    case TVS_ENOMEM: return "out of device memory or HBM budget";
    case TVS_EDEVICE: return "HIP device error";
    case TVS_ESTATE: return "call out of order";
    case TVS_ERANGE: return "index, size or value out of range";
    default: return "unknown status";
    }
}

const char *tvs_last_error(tvs_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

void tvs_destroy(tvs_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->cfg.device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->fill_stream) (void)hipStreamSynchronize(ctx->fill_stream);
    free_histories(ctx);
    free_batch(ctx);
    dfree(ctx, &ctx->x0, (size_t)ctx->nvox);
    dfree(ctx, &ctx->x, (size_t)ctx->nvox);
    dfree(ctx, &ctx->xio, (size_t)ctx->nvox);
    dfree(ctx, &ctx->g, (size_t)ctx->nvox);
    dfree(ctx, &ctx->flags, (size_t)kNumFlags);
    dfree(ctx, &ctx->dot, (size_t)(3 * (int64_t)ctx->cfg.block_size));
    dfree(ctx, &ctx->part, (size_t)ctx->nparts);
    dfree(ctx, &ctx->scal, (size_t)4);
    dfree(ctx, &ctx->ticket, (size_t)4);
    dfree(ctx, &ctx->sched, (size_t)1);
    dfree(ctx, &ctx->dlog, (size_t)kDevLogCap);
    dfree(ctx, &ctx->cpart, (size_t)tvs::tv_check_parts(ctx->gd));
    if (ctx->ev_sched) (void)hipEventDestroy(ctx->ev_sched);
    for (auto &e : ctx->tev)
        if (e) (void)hipEventDestroy(e);
    for (int q = 0; q < kChunkBuffers; q++) {
        if (ctx->ev_filled[q]) (void)hipEventDestroy(ctx->ev_filled[q]);
        if (ctx->ev_free[q]) (void)hipEventDestroy(ctx->ev_free[q]);
        if (ctx->bev_filled[q]) (void)hipEventDestroy(ctx->bev_filled[q]);
        if (ctx->bev_free[q]) (void)hipEventDestroy(ctx->bev_free[q]);
    }
    if (ctx->bev_fork) (void)hipEventDestroy(ctx->bev_fork);
    if (ctx->fill_stream) (void)hipStreamDestroy(ctx->fill_stream);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

int tvs_create(const tvs_grid *grid, const tvs_config *cfg_in, tvs_ctx **out)
{
    tvs_ctx *ctx = nullptr;
    if (!out) return TVS_EINVAL;
    *out = nullptr;
    if (!grid) return TVS_EINVAL;
    tvs_config cfg;
    if (cfg_in) cfg = *cfg_in;
    else tvs_config_default(&cfg);
    if (grid->nx <= 0 || grid->ny <= 0 || grid->nz <= 0) return TVS_EINVAL;
    if (!finite_pos(grid->vx) || !finite_pos(grid->vy) || !finite_pos(grid->vz)) return TVS_EINVAL;
    if (!std::isfinite(grid->ox) || !std::isfinite(grid->oy) || !std::isfinite(grid->oz))
        return TVS_EINVAL;
    if (grid->nx >= (1 << 20) || grid->ny >= (1 << 20) || grid->nz >= (1 << 20)) return TVS_EINVAL;
    const tvs::GridDev gdev = tvs::make_grid_dev(*grid);
    const int64_t nimg = (int64_t)grid->nx * grid->ny * grid->nz;
    const int64_t nvox = tvs::padded_voxels(gdev);     // device image words (tiled layout)
    if (nvox >= ((int64_t)1 << 31)) return TVS_EINVAL;
    if (cfg.block_size < 1 || cfg.block_size > (1 << 24)) return TVS_EINVAL;
    if (cfg.path_mode < 0 || cfg.path_mode > 3) return TVS_EINVAL;
    // the fixed-point store keeps at least 4 code bits in each tag
    if (cfg.path_mode == TVS_PATH_STORE_Q16 && cfg.block_size > (1 << 20)) return TVS_EINVAL;
    if (!std::isfinite(cfg.mlp_step_mm)) return TVS_EINVAL;
    if (cfg.chunk_histories < 0 || cfg.max_tries < 0) return TVS_EINVAL;
    if (cfg.sweep_kernel < 0 || cfg.sweep_kernel > 2) return TVS_EINVAL;
    if (cfg.tile_threads != 0 && cfg.tile_threads != 64 && cfg.tile_threads != 128 &&
        cfg.tile_threads != 256)
        return TVS_EINVAL;
    if (cfg.time_sample < 0) return TVS_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg.device < 0 || cfg.device >= ndev)
        return TVS_EDEVICE;
    if (hipSetDevice(cfg.device) != hipSuccess) return TVS_EDEVICE;
    fbp_scratch_setup(cfg.device);

    ctx = new tvs_ctx();
    ctx->grid = *grid;
    ctx->cfg = cfg;
    ctx->gd = gdev;
    ctx->nimg = nimg;
    ctx->nvox = nvox;
    ctx->ntiles = tvs::num_tiles(gdev);
    double step = cfg.mlp_step_mm > 0.0 ? cfg.mlp_step_mm : std::min(grid->vx, grid->vy);
    ctx->mlp = tvs::MlpCfg{step, cfg.mlp_log_term ? 1 : 0, cfg.mlp_const_power ? 1 : 0};
    if (ctx->cfg.max_tries == 0) ctx->cfg.max_tries = 100000;
    ctx->split = (cfg.sweep_kernel == 2) ? 1 : 0;
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cfg.device) !=
            hipSuccess)
            cus = 0;
        const int per_cu = cfg.fill_wgs_per_cu;
        ctx->fill_wgs = (per_cu > 0 && cus > 0) ? (int64_t)per_cu * cus : 0;
        // the library's choice: about 40 % of the chunks at full occupancy
        // (within a few % of the best share at 200x200x16 and 256x256x32;
        // tvs_autotune times the shares on the loaded histories)
        ctx->fill_wide_pct = cfg.fill_wide_pct < 0 ? 40 : std::min(cfg.fill_wide_pct, 100);
        // Tile workgroup size: 128 lanes on the fly (they leave the row
        // formation beside the DROP chain more room) and for grids of more
        // tiles than twice the 256-lane workgroups the device holds at once
        // (8 per CU: fewer rounds of workgroups per step); else 256 lanes,
        // with which a step of a path store is shortest
        const int64_t resident256 = 8 * (int64_t)(cus > 0 ? cus : 256);
        const bool small = cfg.path_mode == TVS_PATH_ON_THE_FLY || ctx->ntiles > 2 * resident256;
        ctx->threads = cfg.tile_threads ? cfg.tile_threads : (small ? 128 : 256);
    }

    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) {
        delete ctx;
        return TVS_EDEVICE;
    }
    ctx->budget = cfg.hbm_budget_bytes ? cfg.hbm_budget_bytes : (uint64_t)(0.8 * (double)freeb);

    int rc = TVS_OK;
    ctx->nparts = tvs::tv_num_parts(ctx->gd);
    if (!rc) rc = dalloc(ctx, &ctx->x, (size_t)nvox);
    if (!rc) rc = dalloc(ctx, &ctx->x0, (size_t)nvox);
    if (!rc) rc = dalloc(ctx, &ctx->xio, (size_t)nvox);
    if (!rc) rc = dalloc(ctx, &ctx->g, (size_t)nvox);
    if (!rc) rc = dalloc(ctx, &ctx->flags, (size_t)kNumFlags);
    if (!rc) rc = dalloc(ctx, &ctx->dot, (size_t)(3 * (int64_t)cfg.block_size));
    if (!rc) rc = dalloc(ctx, &ctx->part, (size_t)ctx->nparts);
    if (!rc) rc = dalloc(ctx, &ctx->scal, (size_t)4);
    if (!rc) rc = dalloc(ctx, &ctx->ticket, (size_t)4);
    if (!rc) rc = dalloc(ctx, &ctx->sched, (size_t)1);
    if (!rc) rc = dalloc(ctx, &ctx->dlog, (size_t)kDevLogCap);
    if (!rc) rc = dalloc(ctx, &ctx->cpart, (size_t)tvs::tv_check_parts(ctx->gd));
    if (rc) {
        tvs_destroy(ctx);
        return rc;
    }
    if (hipEventCreateWithFlags(&ctx->ev_sched, hipEventDisableTiming) != hipSuccess) {
        tvs_destroy(ctx);
        return TVS_EDEVICE;
    }
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->fill_stream, hipStreamNonBlocking) != hipSuccess) {
        tvs_destroy(ctx);
        return TVS_EDEVICE;
    }
    for (int q = 0; q < kChunkBuffers; q++) {
        if (hipEventCreateWithFlags(&ctx->ev_filled[q], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->ev_free[q], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->bev_filled[q], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->bev_free[q], hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(ctx->ev_free[q], ctx->stream) != hipSuccess) {
            tvs_destroy(ctx);
            return TVS_EDEVICE;
        }
    }
    if (hipEventCreateWithFlags(&ctx->bev_fork, hipEventDisableTiming) != hipSuccess) {
        tvs_destroy(ctx);
        return TVS_EDEVICE;
    }
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemsetAsync(ctx->x, 0, sizeof(double) * nvox, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->x0, 0, sizeof(double) * nvox, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->g, 0, sizeof(double) * nvox, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->flags, 0, sizeof(uint32_t) * kNumFlags, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->ticket, 0, sizeof(uint32_t) * 4, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->scal, 0, sizeof(double) * 4, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        tvs_destroy(ctx);
        return TVS_EDEVICE;
    }
    *out = ctx;
    return TVS_OK;
}

int tvs_load_histories(tvs_ctx *ctx, int64_t n, const tvs_histories *h, int on_device, void *stream)
{
    if (!ctx) return TVS_EINVAL;
    ctx->err.clear();
    if (n < 0) return fail(ctx, TVS_EINVAL, "n must be >= 0");
    if (n >= ((int64_t)1 << 31)) return fail(ctx, TVS_EINVAL, "at most 2^31 - 1 histories");
    if (n > 0 && !h) return fail(ctx, TVS_EINVAL, "histories is NULL");
    const float *src[kNumStreams] = {};
    if (n > 0) {
        const float *tmp[kNumStreams] = {h->ex,  h->ey,  h->ez, h->qx, h->qy, h->qz, h->eth,
                                         h->eps, h->qth, h->qps, h->ux, h->uy, h->wepl};
        for (int q = 0; q < kNumStreams; q++) {
            if (!tmp[q]) return fail(ctx, TVS_EINVAL, "a history stream is NULL");
            src[q] = tmp[q];
        }
    }
    HIPCHK(hipSetDevice(ctx->cfg.device));
    hipStream_t st = pick(ctx, stream);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->fill_stream));
    free_histories(ctx);
    reset_state(ctx);
    HIPCHK(hipMemsetAsync(ctx->x, 0, sizeof(double) * ctx->nvox, st));
    HIPCHK(hipMemsetAsync(ctx->x0, 0, sizeof(double) * ctx->nvox, st));
    HIPCHK(hipMemsetAsync(ctx->flags, 0, sizeof(uint32_t) * kNumFlags, st));
    ctx->batch.valid = false;
    ctx->nh = n;

    int rc = dalloc(ctx, &ctx->hist, (size_t)(kNumStreams * n));
    if (!rc) rc = dalloc(ctx, &ctx->row_off, (size_t)(n + 1));
    if (!rc) rc = dalloc(ctx, &ctx->norm2, (size_t)n);
    if (!rc) rc = dalloc(ctx, &ctx->seg_off, (size_t)(n + 1));
    if (rc) {
        free_histories(ctx);
        return rc;
    }
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    for (int q = 0; q < kNumStreams && n > 0; q++) {
        hipError_t e = hipMemcpyAsync(ctx->hist + q * n, src[q], sizeof(float) * n, kind, st);
        if (e != hipSuccess) {
            free_histories(ctx);
            return fail(ctx, TVS_EDEVICE, std::string("history copy: ") + hipGetErrorString(e));
        }
    }
    // validation on the device (the inputs may live there already)
    uint32_t bad = 0, jmax = 0;
    {
        hipError_t e = tvs::launch_validate(hist_dev(ctx), n, ctx->mlp.step,
                                            ctx->flags + kFlagInvalid, ctx->flags + kFlagJmax, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&bad, ctx->flags + kFlagInvalid, sizeof(uint32_t),
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&jmax, ctx->flags + kFlagJmax, sizeof(uint32_t),
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            free_histories(ctx);
            return fail(ctx, TVS_EDEVICE, std::string("validation: ") + hipGetErrorString(e));
        }
    }
    if (bad) {
        free_histories(ctx);
        (void)hipMemsetAsync(ctx->flags, 0, sizeof(uint32_t) * kNumFlags, st);
        return fail(ctx, TVS_EINVAL,
                    std::to_string(bad) + " histories hold NaN/inf, |value| > 1e6, a zero beam "
                                          "axis or more than 2^20 MLP vertices");
    }
    // entry-side MLP table for every vertex depth of these histories
    if (jmax > 0) {
        rc = dalloc(ctx, &ctx->s1i, (size_t)(3 * (int64_t)jmax));
        if (!rc) {
            ctx->nj = jmax;
            hipError_t e = tvs::launch_mlp_table(ctx->mlp, ctx->nj, ctx->s1i, st);
            if (e != hipSuccess) rc = fail(ctx, TVS_EDEVICE, std::string("MLP table: ") + hipGetErrorString(e));
            ctx->mlp.s1i = ctx->s1i;
            ctx->mlp.nj = ctx->nj;
            ctx->mlp.err = ctx->flags + kFlagLists;
        }
        if (rc) {
            std::string msg = ctx->err;
            free_histories(ctx);
            return fail(ctx, rc, msg);
        }
    }
    // the tile lists of every block (their layout; rows themselves are
    // formed now for a path store, per chunk and sweep otherwise)
    rc = build_tile_lists(ctx, st);
    if (!rc) rc = form_entries(ctx, st);
    if (rc) {
        std::string msg = ctx->err;
        free_histories(ctx);
        return fail(ctx, rc, msg);
    }
    ctx->loaded = true;
    ctx->timed = false;
    ctx->spans.clear();
    return TVS_OK;
}

int tvs_set_image(tvs_ctx *ctx, const float *x0, int on_device, void *stream)
{
    if (!ctx) return TVS_EINVAL;
    ctx->err.clear();
    if (!x0) return fail(ctx, TVS_EINVAL, "image is NULL");
    HIPCHK(hipSetDevice(ctx->cfg.device));
    hipStream_t st = pick(ctx, stream);
    if (!on_device) {
        for (int64_t j = 0; j < ctx->nimg; j++)
            if (!std::isfinite(x0[j])) return fail(ctx, TVS_EINVAL, "image holds NaN/inf");
    }
    HIPCHK(hipMemcpyAsync(ctx->xio, x0, sizeof(float) * ctx->nimg,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    HIPCHK(tvs::launch_widen(ctx->gd, ctx->xio, ctx->x, st));
    HIPCHK(hipMemcpyAsync(ctx->x0, ctx->x, sizeof(double) * ctx->nvox, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemsetAsync(ctx->flags + kFlagRange, 0, sizeof(uint32_t), st));
    if (!on_device) HIPCHK(hipStreamSynchronize(st));
    reset_state(ctx);
    ctx->batch.valid = false;
    return TVS_OK;
}

}  // extern "C"

namespace {

// Checks the FBP parameters against the context and sizes the bins: lateral
// bin width tau, nt lateral bins (2 ceil(R / tau) + 2, R the farthest slice
// corner from the axis), nb = A * nz * nt bins.
int fbp_geometry(tvs_ctx *ctx, const tvs_fbp_params *p, const char *who, double &tau,
                 int32_t &nt, int64_t &nb)
{
    if (!p) return fail(ctx, TVS_EINVAL, "params is NULL");
    if (p->n_angles < 1) return fail(ctx, TVS_EINVAL, "n_angles must be >= 1");
    if (!(p->t_bin_mm >= 0.0) || !std::isfinite(p->t_bin_mm))
        return fail(ctx, TVS_EINVAL, "t_bin_mm must be finite and >= 0");
    if (p->median_radius < 0 || p->median_radius > 2)
        return fail(ctx, TVS_EINVAL, "median_radius must lie in 0..2");
    if (!ctx->loaded) return fail(ctx, TVS_ESTATE, std::string(who) + " before tvs_load_histories");
    const tvs_grid &g = ctx->grid;
    tau = p->t_bin_mm > 0.0 ? p->t_bin_mm : g.vx;
    double R = 0.0;
    for (int cx = 0; cx < 2; cx++)
        for (int cy = 0; cy < 2; cy++)
            R = std::max(R, std::hypot(g.ox + cx * g.nx * g.vx, g.oy + cy * g.ny * g.vy));
    const double ntd = 2.0 * std::ceil(R / tau) + 2.0;
    if (!(ntd <= 16777216.0)) return fail(ctx, TVS_EINVAL, "t_bin_mm too small for the grid");
    nt = (int32_t)ntd;
    nb = (int64_t)p->n_angles * g.nz * nt;
    return TVS_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

int tvs_initial_fbp(tvs_ctx *ctx, const tvs_fbp_params *p, float *out, int on_device, void *stream)
{
    if (!ctx) return TVS_EINVAL;
    ctx->err.clear();
    double tau = 0.0;
    int32_t nt = 0;
    int64_t nb = 0;
    int rc = fbp_geometry(ctx, p, "tvs_initial_fbp", tau, nt, nb);
    if (rc) return rc;
    HIPCHK(hipSetDevice(ctx->cfg.device));
    hipStream_t st = pick(ctx, stream);
    const tvs_grid &g = ctx->grid;
    const int32_t A = p->n_angles;

    unsigned long long *sum = nullptr;
    uint32_t *cnt = nullptr;
    double *pb = nullptr, *qb = nullptr, *cs = nullptr, *img = nullptr;
    auto release = [&]() {
        dfree(ctx, &sum, (size_t)nb);
        dfree(ctx, &cnt, (size_t)nb);
        dfree(ctx, &pb, (size_t)nb);
        dfree(ctx, &qb, (size_t)nb);
        dfree(ctx, &cs, (size_t)(2 * A));
        dfree(ctx, &img, (size_t)ctx->nimg);
    };
    rc = dalloc(ctx, &sum, (size_t)nb);
    if (!rc) rc = dalloc(ctx, &cnt, (size_t)nb);
    if (!rc) rc = dalloc(ctx, &pb, (size_t)nb);
    if (!rc) rc = dalloc(ctx, &qb, (size_t)nb);
    if (!rc) rc = dalloc(ctx, &cs, (size_t)(2 * A));
    if (!rc) rc = dalloc(ctx, &img, (size_t)ctx->nimg);
    if (rc) {
        release();
        return rc;
    }
    // cos, sin of every beam angle a * 2 pi / A
    std::vector<double> tab((size_t)(2 * A));
    const double da = 2.0 * 3.14159265358979323846 / (double)A;
    for (int32_t a = 0; a < A; a++) {
        const double phi = (double)a * da;
        tab[(size_t)(2 * a)] = std::cos(phi);
        tab[(size_t)(2 * a + 1)] = std::sin(phi);
    }
    hipError_t e = hipMemsetAsync(sum, 0, sizeof(unsigned long long) * nb, st);
    if (e == hipSuccess) e = hipMemsetAsync(cnt, 0, sizeof(uint32_t) * nb, st);
    if (e == hipSuccess) e = hipMemcpyAsync(cs, tab.data(), sizeof(double) * 2 * A, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = tvs::launch_fbp_bin(ctx->gd, hist_dev(ctx), ctx->nh, A, tau, nt, sum, cnt, st);
    if (e == hipSuccess) e = tvs::launch_fbp_mean(sum, cnt, nb, pb, st);
    if (e == hipSuccess) e = tvs::launch_fbp_filter(pb, (int64_t)A * g.nz, nt, tau, qb, st);
    if (e == hipSuccess)
        e = tvs::launch_fbp_backproject(ctx->gd, qb, cs, A, tau, nt, p->clip_negative ? 1 : 0, img, st);
    if (e == hipSuccess) e = tvs::launch_median(ctx->gd, img, p->median_radius, ctx->xio, st);
    // the result becomes the context image, as by tvs_set_image
    if (e == hipSuccess) e = tvs::launch_widen(ctx->gd, ctx->xio, ctx->x, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->x0, ctx->x, sizeof(double) * ctx->nvox, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->flags + kFlagRange, 0, sizeof(uint32_t), st);
    if (e == hipSuccess && out)
        e = hipMemcpyAsync(out, ctx->xio, sizeof(float) * ctx->nimg,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    release();
    if (e != hipSuccess) return fail(ctx, TVS_EDEVICE, std::string("initial fbp: ") + hipGetErrorString(e));
    reset_state(ctx);
    ctx->batch.valid = false;
    return TVS_OK;
}

int tvs_initial_fbp_noalloc(tvs_ctx *ctx, const tvs_fbp_params *p, float *out, int on_device,
                            void *stream)
{
    if (!ctx) return TVS_EINVAL;
    ctx->err.clear();
    double tau = 0.0;
    int32_t nt = 0;
    int64_t nb = 0;
    int rc = fbp_geometry(ctx, p, "tvs_initial_fbp_noalloc", tau, nt, nb);
    if (rc) return rc;
    const int32_t A = p->n_angles;
    // workspace layout: bin sums and counts (cleared), mean and filtered
    // projections, angle table, backprojected image; each part 256-aligned
    const size_t o_sum = 0;
    const size_t o_cnt = o_sum + align256(sizeof(unsigned long long) * (size_t)nb);
    const size_t o_pb = o_cnt + align256(sizeof(uint32_t) * (size_t)nb);
    const size_t o_qb = o_pb + align256(sizeof(double) * (size_t)nb);
    const size_t o_cs = o_qb + align256(sizeof(double) * (size_t)nb);
    const size_t o_img = o_cs + align256(sizeof(double) * 2 * (size_t)A);
    const size_t need = o_img + align256(sizeof(double) * (size_t)ctx->nimg);
    if (need > kFbpScratchBytes)
        return fail(ctx, TVS_ERANGE,
                    "tvs_initial_fbp_noalloc needs " + std::to_string(need) +
                        " B of workspace (" + std::to_string(nb) + " bins, " +
                        std::to_string(ctx->nimg) + " voxels); its fixed workspace holds " +
                        std::to_string(kFbpScratchBytes) + " B");
    const int dev = ctx->cfg.device;
    if (dev < 0 || dev >= kMaxDevices)
        return fail(ctx, TVS_EDEVICE, "device ordinal beyond the workspace table");
    HIPCHK(hipSetDevice(dev));
    fbp_scratch_setup(dev);
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev])
            return fail(ctx, TVS_EDEVICE,
                        std::string("workspace address lookup failed: ") +
                            hipGetErrorString(g_scratch_status[dev]));
        base = static_cast<unsigned char *>(g_scratch_ptr[dev]);
    }
    hipStream_t st = pick(ctx, stream);
    auto *sum = reinterpret_cast<unsigned long long *>(base + o_sum);
    auto *cnt = reinterpret_cast<uint32_t *>(base + o_cnt);
    auto *pb = reinterpret_cast<double *>(base + o_pb);
    auto *qb = reinterpret_cast<double *>(base + o_qb);
    auto *cs = reinterpret_cast<double *>(base + o_cs);
    auto *img = reinterpret_cast<double *>(base + o_img);
    const tvs_grid &g = ctx->grid;
    // sums and counts start at zero (a fill kernel: the workspace keeps the
    // previous call's contents)
    hipError_t e = tvs::launch_zero_i64(reinterpret_cast<long long *>(base + o_sum),
                                        (int64_t)(o_pb / sizeof(long long)), st);
    if (e == hipSuccess) e = tvs::launch_fbp_angles(A, cs, st);
    if (e == hipSuccess) e = tvs::launch_fbp_bin(ctx->gd, hist_dev(ctx), ctx->nh, A, tau, nt, sum, cnt, st);
    if (e == hipSuccess) e = tvs::launch_fbp_mean(sum, cnt, nb, pb, st);
    if (e == hipSuccess) e = tvs::launch_fbp_filter(pb, (int64_t)A * g.nz, nt, tau, qb, st);
    if (e == hipSuccess)
        e = tvs::launch_fbp_backproject(ctx->gd, qb, cs, A, tau, nt, p->clip_negative ? 1 : 0, img, st);
    if (e == hipSuccess) e = tvs::launch_median(ctx->gd, img, p->median_radius, ctx->xio, st);
    if (e == hipSuccess) e = tvs::launch_widen(ctx->gd, ctx->xio, ctx->x, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->x0, ctx->x, sizeof(double) * ctx->nvox, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
        e = tvs::launch_set_counter(reinterpret_cast<int32_t *>(ctx->flags + kFlagRange), 0, st);
    if (e == hipSuccess && out)
        e = hipMemcpyAsync(out, ctx->xio, sizeof(float) * ctx->nimg,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && out && !on_device) e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return fail(ctx, TVS_EDEVICE, std::string("initial fbp (no-alloc): ") + hipGetErrorString(e));
    reset_state(ctx);
    ctx->batch.valid = false;
    return TVS_OK;
}

int tvs_hull_detect(tvs_ctx *ctx, const tvs_hull_params *p, uint8_t *hull, int on_device,
                    void *stream)
{
    if (!ctx) return TVS_EINVAL;
    ctx->err.clear();
    if (!p) return fail(ctx, TVS_EINVAL, "params is NULL");
    if (p->min_in < 0 || p->max_out < 0) return fail(ctx, TVS_EINVAL, "min_in and max_out must be >= 0");
    if (std::isnan(p->wepl_in_mm) || std::isnan(p->wepl_out_mm))
        return fail(ctx, TVS_EINVAL, "WEPL thresholds must not be NaN");
    if (!ctx->loaded) return fail(ctx, TVS_ESTATE, "tvs_hull_detect before tvs_load_histories");
    HIPCHK(hipSetDevice(ctx->cfg.device));
    hipStream_t st = pick(ctx, stream);
    uint32_t *cnt = nullptr;
    uint8_t *hd = nullptr;
    int rc = dalloc(ctx, &cnt, (size_t)(2 * ctx->nvox));
    if (!rc) rc = dalloc(ctx, &hd, (size_t)ctx->nimg);
    if (rc) {
        dfree(ctx, &cnt, (size_t)(2 * ctx->nvox));
        return rc;
    }
    // the counting threshold -inf when space modelling is off makes every
    // line count; min_in = 0 then accepts every voxel on that side
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(uint32_t) * 2 * ctx->nvox, st);
    if (e == hipSuccess)
        e = tvs::launch_hull_counts(ctx->gd, hist_dev(ctx), ctx->nh, p->wepl_in_mm, p->wepl_out_mm,
                                    cnt, cnt + ctx->nvox, (uint32_t)p->min_in,
                                    (uint32_t)p->max_out + 1u, st);
    if (e == hipSuccess)
        e = tvs::launch_hull_decide(ctx->gd, cnt, cnt + ctx->nvox, (uint32_t)p->min_in,
                                    (uint32_t)p->max_out, hd, p->mask_image ? ctx->x : nullptr, st);
    if (e == hipSuccess && p->mask_image)
        e = hipMemcpyAsync(ctx->x0, ctx->x, sizeof(double) * ctx->nvox, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && hull)
        e = hipMemcpyAsync(hull, hd, (size_t)ctx->nimg,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dfree(ctx, &cnt, (size_t)(2 * ctx->nvox));
    dfree(ctx, &hd, (size_t)ctx->nimg);
    if (e != hipSuccess) return fail(ctx, TVS_EDEVICE, std::string("hull: ") + hipGetErrorString(e));
    if (p->mask_image) {
        reset_state(ctx);
        ctx->batch.valid = false;
    }
    return TVS_OK;
}

int tvs_iterate(tvs_ctx *ctx, const tvs_params *p, int32_t K, void *stream)
{
    if (!ctx) return TVS_EINVAL;
    ctx->err.clear();
    int rc = validate_params(ctx, p);
    if (rc) return rc;
    if (K < 0) return fail(ctx, TVS_EINVAL, "K must be >= 0");
    if (!ctx->loaded) return fail(ctx, TVS_ESTATE, "tvs_iterate before tvs_load_histories");
    HIPCHK(hipSetDevice(ctx->cfg.device));
    hipStream_t st = pick(ctx, stream);
    tvs::TvBuffers tb = tv_bufs(ctx);
    if (!ctx->seeded) {
        ctx->rng = p->seed;
        ctx->seeded = true;
    }
    const bool checked = (p->variant == TVS_OTVS) || (p->variant == TVS_NTVS && p->tv_check);
    const int32_t nsteps = (p->variant == TVS_OTVS) ? 1 : p->N;
    // unchecked steps take ell from the host: bring a device-held schedule back
    if (!checked) {
        rc = settle_sched(ctx);
        if (rc) return rc;
    }
    if (K > 0) {
        ctx->tev_used = 0;
        ctx->spans.clear();
        ctx->timed = true;
    }
    const tvs::CheckBuffers cb{ctx->cpart, ctx->ticket + 1, ctx->scal + 2};
    const double check_alpha = (p->variant == TVS_OTVS) ? 0.5 : p->alpha;
    if (checked && K > 0 && !ctx->dev_sched) {
        HIPCHK(tvs::launch_sched_set(ctx->sched, ctx->ell, ctx->rng, st));
        ctx->dev_sched = true;
    }
    for (int32_t kk = 0; kk < K; kk++) {
        const int64_t k = ctx->k;
        if (checked && ctx->dlog_n + nsteps > kDevLogCap) {
            // the record buffer is full: copy it back and go on
            HIPCHK(hipEventRecord(ctx->ev_sched, st));
            rc = settle_sched(ctx);
            if (rc) return rc;
            HIPCHK(tvs::launch_sched_set(ctx->sched, ctx->ell, ctx->rng, st));
            ctx->dev_sched = true;
        }
        if (p->variant == TVS_NTVS) {
            if (checked) HIPCHK(tvs::launch_sched_draw(ctx->sched, k, st));
            else ctx->ell = draw_ell(k, ctx->ell, ctx->rng);
        }
        const long c0 = mark(ctx, st);
        for (int32_t n = 0; n < nsteps; n++) {
            HIPCHK(tvs::launch_tv_grad(ctx->gd, ctx->x, p->tv_eps, tb, st));
            if (!checked) {
                tvs_step_log rec;
                std::memset(&rec, 0, sizeof(rec));
                rec.k = (int32_t)k;
                rec.n = n;
                rec.ell_start = ctx->ell;
                rec.gnorm = -1.0;
                double beta = (p->variant == TVS_DECOUPLED)
                                  ? std::pow(p->alpha, (double)(n + 1)) * std::pow(p->gamma, (double)k)
                                  : std::pow(p->alpha, (double)ctx->ell);
                HIPCHK(tvs::launch_tv_step(ctx->gd, ctx->x, beta, tb, st));
                ctx->ell += 1;
                rec.tries = 1;
                rec.accepted = 1;
                ctx->tries += 1;
                ctx->log.push_back(rec);
            } else {
                // decided on the device: no host round trip
                HIPCHK(tvs::launch_tv_check(ctx->gd, ctx->x, p->tv_eps, check_alpha,
                                            ctx->cfg.max_tries, (int32_t)k, n, ctx->sched,
                                            ctx->dlog + ctx->dlog_n, cb, tb, st));
                HIPCHK(tvs::launch_tv_apply(ctx->gd, ctx->x, tb, cb, st));
                ctx->dlog_n += 1;
            }
        }
        const long c1 = mark(ctx, st);
        span(ctx, 0, c0, c1);
        rc = run_sweep(ctx, p->lambda, st);
        if (rc) return rc;
        span(ctx, 1, c1, mark(ctx, st));
        ctx->k += 1;
    }
    if (checked && K > 0) HIPCHK(hipEventRecord(ctx->ev_sched, st));
    return TVS_OK;
}

int tvs_get_image(tvs_ctx *ctx, float *out, int on_device, void *stream)
{
    if (!ctx) return TVS_EINVAL;
    ctx->err.clear();
    if (!out) return fail(ctx, TVS_EINVAL, "output is NULL");
    HIPCHK(hipSetDevice(ctx->cfg.device));
    hipStream_t st = pick(ctx, stream);
    int rc = check_flags(ctx, st);
    if (rc) return rc;
    HIPCHK(tvs::launch_narrow(ctx->gd, ctx->x, ctx->xio, st));
    HIPCHK(hipMemcpyAsync(out, ctx->xio, sizeof(float) * ctx->nimg,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    if (!on_device) HIPCHK(hipStreamSynchronize(st));
    return TVS_OK;
}

int tvs_get_stats(tvs_ctx *ctx, tvs_stats *out)
{
    if (!ctx || !out) return TVS_EINVAL;
    ctx->err.clear();
    HIPCHK(hipSetDevice(ctx->cfg.device));
    int src = settle_sched(ctx);
    if (src) return src;
    if (ctx->timed && !ctx->spans.empty()) {
        HIPCHK(hipEventSynchronize(ctx->tev[ctx->spans.back().b]));
        HIPCHK(hipStreamSynchronize(ctx->fill_stream));
        for (int q = 0; q < 6; q++) {
            ctx->tot_ms[q] = 0.0;
            ctx->tot_n[q] = 0;
        }
        double last[4] = {0, 0, 0, 0};
        size_t last_cycle_start = 0;
        for (const auto &sp : ctx->spans) {
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, ctx->tev[sp.a], ctx->tev[sp.b]));
            ctx->tot_ms[sp.kind] += ms;
            ctx->tot_n[sp.kind] += 1;
            if (sp.kind == 0) {
                last_cycle_start = sp.a;
                last[0] = ms;
                last[2] = 0;
            } else if (sp.kind == 1) {
                last[1] = ms;
            } else if (sp.kind == 2 && sp.a >= last_cycle_start) {
                last[2] += ms;
            }
        }
        ctx->last_tv_ms = last[0];
        ctx->last_sweep_ms = last[1];
        ctx->last_rows_ms = last[2];
        ctx->timed = false;
    }
    int rc = check_flags(ctx, ctx->stream);
    if (rc) return rc;
    out->k = ctx->k;
    out->ell = ctx->ell;
    out->n_hist = ctx->nh;
    out->n_skipped = ctx->skipped;
    out->nnz = ctx->nnz;
    out->steps = (int64_t)ctx->log.size();
    out->tries = ctx->tries;
    out->max_row_nnz = ctx->max_row;
    out->last_sweep_ms = ctx->last_sweep_ms;
    out->last_tv_ms = ctx->last_tv_ms;
    out->last_rows_ms = ctx->last_rows_ms;
    out->device_bytes = ctx->bytes;
    out->tv_ms_total = ctx->tot_ms[0];
    out->sweep_ms_total = ctx->tot_ms[1];
    out->rows_ms_total = ctx->tot_ms[2];
    out->drop_ms_total = ctx->tot_ms[3];
    out->cycles_timed = ctx->tot_n[1];
    out->rows_launches = ctx->tot_n[2];
    out->drop_launches = ctx->tot_n[3];
    out->k1_ms_total = ctx->tot_ms[4];
    out->k2_ms_total = ctx->tot_ms[5];
    out->k_samples = ctx->tot_n[4];
    out->batch_ms_total = ctx->batch.ms_total;
    out->batch_cycles = ctx->batch.cycles;
    out->batch_size = ctx->batch.valid ? ctx->batch.S : 0;
    out->pad = 0;
    return TVS_OK;
}

int tvs_get_step_log(tvs_ctx *ctx, tvs_step_log *out, int64_t cap, int64_t *n)
{
    if (!ctx || !n || cap < 0 || (cap > 0 && !out)) return TVS_EINVAL;
    ctx->err.clear();
    HIPCHK(hipSetDevice(ctx->cfg.device));
    int rc = settle_sched(ctx);
    if (rc) return rc;
    *n = (int64_t)ctx->log.size();
    int64_t m = std::min<int64_t>(cap, *n);
    if (m > 0) std::memcpy(out, ctx->log.data(), sizeof(tvs_step_log) * (size_t)m);
    return TVS_OK;
}

int tvs_debug_rows(tvs_ctx *ctx, int64_t first, int64_t count, int64_t *row_nnz, int32_t *idx,
                   float *chord, float *norm2, int64_t cap)
{
    if (!ctx) return TVS_EINVAL;
    ctx->err.clear();
    if (!ctx->loaded) return fail(ctx, TVS_ESTATE, "no histories loaded");
    if (first < 0 || count < 0 || first + count > ctx->nh)
        return fail(ctx, TVS_ERANGE, "history range outside the loaded histories");
    if (count > 0 && (!row_nnz || !norm2)) return fail(ctx, TVS_EINVAL, "output is NULL");
    if (count == 0) return TVS_OK;
    HIPCHK(hipSetDevice(ctx->cfg.device));
    hipStream_t st = ctx->stream;
    int64_t *off = nullptr;
    int rc = dalloc(ctx, &off, (size_t)(count + 1));
    if (rc) return rc;
    rc = count_rows(ctx, first, count, off, st);
    std::vector<int64_t> offh((size_t)count + 1);
    if (!rc && hipMemcpy(offh.data(), off, sizeof(int64_t) * (count + 1), hipMemcpyDeviceToHost) !=
                   hipSuccess)
        rc = fail(ctx, TVS_EDEVICE, "row offsets copy");
    if (rc) {
        dfree(ctx, &off, (size_t)(count + 1));
        return rc;
    }
    const int64_t tot = offh[(size_t)count];
    for (int64_t q = 0; q < count; q++) row_nnz[q] = offh[(size_t)q + 1] - offh[(size_t)q];
    if (tot > cap || (tot > 0 && (!idx || !chord))) {
        dfree(ctx, &off, (size_t)(count + 1));
        return fail(ctx, TVS_ERANGE, "cap smaller than the entries of the requested rows");
    }
    int32_t *di = nullptr;
    float *dc = nullptr, *dn = nullptr;
    rc = dalloc(ctx, &di, (size_t)std::max<int64_t>(tot, 1));
    if (!rc) rc = dalloc(ctx, &dc, (size_t)std::max<int64_t>(tot, 1));
    if (!rc) rc = dalloc(ctx, &dn, (size_t)count);
    if (!rc) {
        RowSet rs;
        rs.first = first;
        rs.n = count;
        rs.base = 0;
        rs.row_off = off;
        rs.idx = di;
        rs.chord32 = dc;
        rs.norm2 = dn;
        hipError_t e = tvs::launch_rows_fill(ctx->gd, hist_dev(ctx), ctx->mlp, rs, st);
        if (e == hipSuccess && tot > 0)
            e = hipMemcpyAsync(idx, di, sizeof(int32_t) * tot, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess) {
            // tiled-layout words to x-fastest voxel indices (the ABI's order)
            const GridDev &g = ctx->gd;
            for (int64_t q = 0; q < tot; q++) {
                int64_t i, j, k;
                tvs::vcoord(g, idx[q], i, j, k);
                idx[q] = (int32_t)((k * g.ny + j) * g.nx + i);
            }
        }
        if (e == hipSuccess && tot > 0)
            e = hipMemcpyAsync(chord, dc, sizeof(float) * tot, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(norm2, dn, sizeof(float) * count, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail(ctx, TVS_EDEVICE, std::string("debug rows: ") + hipGetErrorString(e));
    }
    dfree(ctx, &di, (size_t)std::max<int64_t>(tot, 1));
    dfree(ctx, &dc, (size_t)std::max<int64_t>(tot, 1));
    dfree(ctx, &dn, (size_t)count);
    dfree(ctx, &off, (size_t)(count + 1));
    return rc;
}

}  // extern "C"

namespace {

bool same_params(const tvs_params &a, const tvs_params &b)
{
    return a.lambda == b.lambda && a.N == b.N && a.alpha == b.alpha && a.tv_check == b.tv_check &&
           a.variant == b.variant && a.tv_eps == b.tv_eps && a.seed == b.seed &&
           (a.variant != TVS_DECOUPLED || a.gamma == b.gamma);
}

// (Re)allocates the S-image buffers and starts every setting from x0.
int batch_init(tvs_ctx *ctx, const tvs_params *p, int S, hipStream_t st)
{
    auto &B = ctx->batch;
    if (B.S != S) {
        free_batch(ctx);
        B.S = S;
        const size_t n = (size_t)(ctx->nvox * S);
        int rc = dalloc(ctx, &B.b.x, n);
        if (!rc) rc = dalloc(ctx, &B.b.g, n);
        if (!rc) rc = dalloc(ctx, &B.b.part, (size_t)(tvs::batch_num_parts(ctx->gd, S) * S));
        if (!rc) rc = dalloc(ctx, &B.b.ticket, (size_t)4);
        if (!rc) rc = dalloc(ctx, &B.b.norm2, (size_t)S);
        if (!rc) rc = dalloc(ctx, &B.b.lambda, (size_t)S);
        if (!rc) rc = dalloc(ctx, &B.b.eps, (size_t)S);
        if (!rc) rc = dalloc(ctx, &B.b.cyc, (size_t)4);
        if (!rc) rc = dalloc(ctx, &B.dot, (size_t)(3 * (int64_t)ctx->cfg.block_size * S));
        if (rc) {
            free_batch(ctx);
            return rc;
        }
        B.b.S = S;
        B.b.nvox = ctx->nvox;
        HIPCHK(hipMemsetAsync(B.b.ticket, 0, sizeof(uint32_t) * 4, st));
        HIPCHK(hipMemsetAsync(B.b.g, 0, sizeof(double) * n, st));
    }
    B.p.assign(p, p + S);
    std::vector<double> lam(S), eps(S);
    for (int q = 0; q < S; q++) {
        lam[q] = p[q].lambda;
        eps[q] = p[q].tv_eps;
    }
    HIPCHK(hipMemcpyAsync(B.b.lambda, lam.data(), sizeof(double) * S, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(B.b.eps, eps.data(), sizeof(double) * S, hipMemcpyHostToDevice, st));
    HIPCHK(tvs::launch_replicate(ctx->x0, B.b, st));
    HIPCHK(hipStreamSynchronize(st));
    B.k = 0;
    B.ell.assign(S, 0);
    B.rng.assign(S, 0);
    for (int q = 0; q < S; q++) B.rng[q] = p[q].seed;
    B.valid = true;
    return TVS_OK;
}

// Enqueues the launches of one batched cycle (captured into a graph): the
// TV steps of every setting, then the tile-wise DROP chain for all S
// images.  On the fly, the fill stream joins the capture and forms the
// rows chunk by chunk into the ring of buffers beside the TV steps and the
// chain, with the single-image sweep's filled/free ordering (events of the
// batch's own, so the sweep's events keep their real records); the chain
// waits for the last chunk, which joins the fill stream back.
int batch_cycle(tvs_ctx *ctx, int nmax, hipStream_t st)
{
    auto &Bt = ctx->batch;
    const int S = Bt.S;
    const int64_t B = ctx->cfg.block_size, nb = ctx->nblocks;
    const bool otf = ctx->cfg.path_mode == TVS_PATH_ON_THE_FLY;
    const int64_t step = otf ? ctx->chunk : ctx->nh;
    const int64_t nchunks = nb > 0 ? (ctx->nh + step - 1) / step : 0;
    const int64_t NB = ctx->nbuf;
    hipStream_t fs = ctx->fill_stream;
    auto fill = [&](int64_t c) -> int {
        const int q = chunk_buffer(ctx, c);
        if (c >= NB) HIPCHK(hipStreamWaitEvent(fs, ctx->bev_free[q], 0));
        tvs::TileFill f = chunk_fill(ctx, c, std::min(step, ctx->nh - c * step));
        HIPCHK(tvs::launch_rows_fill_tiled(ctx->gd, hist_dev(ctx), ctx->mlp, f, fs));
        HIPCHK(hipEventRecord(ctx->bev_filled[q], fs));
        return TVS_OK;
    };
    if (otf && nchunks > 0) {
        HIPCHK(hipEventRecord(ctx->bev_fork, st));
        HIPCHK(hipStreamWaitEvent(fs, ctx->bev_fork, 0));
        for (int64_t c = 0; c < std::min<int64_t>(NB, nchunks); c++) {
            int rc = fill(c);
            if (rc) return rc;
        }
    }
    for (int n = 0; n < nmax; n++) {
        uint32_t active = 0;
        for (int q = 0; q < S; q++)
            if (Bt.p[q].N > n) active |= 1u << q;
        HIPCHK(tvs::launch_tvb_grad(ctx->gd, Bt.b, active, st));
        HIPCHK(tvs::launch_tvb_step(Bt.b, active, n, nmax, st));
    }
    if (nb == 0) {
        HIPCHK(tvs::launch_tick(Bt.b.cyc, st));
        return TVS_OK;
    }
    HIPCHK(tvs::launch_zero_i64(Bt.dot, 3 * B * S, st));
    for (int64_t b = 0; b <= nb; b++) {
        const bool has_c = b < nb;
        const int64_t c = has_c ? (b * B) / step : -1;
        const bool first_of_chunk = has_c && (b * B) % step == 0;
        if (otf && first_of_chunk)
            HIPCHK(hipStreamWaitEvent(st, ctx->bev_filled[chunk_buffer(ctx, c)], 0));
        tvs::DropTileArgs A;
        if (b > 0) A.P = block_view(ctx, b - 1, Bt.dot, B * S);
        if (has_c) A.C = block_view(ctx, b, Bt.dot, B * S);
        A.x = Bt.b.x;
        A.big = ctx->big;
        A.dot_max = ctx->dot_max;
        A.zero = Bt.dot + ((b + 1) % 3) * B * S;
        A.B = B;
        A.err = ctx->flags + kFlagRange;
        A.tiles = ctx->act;
        A.nact = ctx->nact;
        HIPCHK(tvs::launch_drop_tiles_batch(A, Bt.b, ctx->ntiles, ctx->bthreads, ctx->bgroup, st));
        if (otf && first_of_chunk && c >= 1 && c - 1 + NB < nchunks) {
            // the launch above was the last to read chunk c - 1's buffer
            HIPCHK(hipEventRecord(ctx->bev_free[chunk_buffer(ctx, c - 1)], st));
            int rc = fill(c - 1 + NB);
            if (rc) return rc;
        }
    }
    HIPCHK(tvs::launch_tick(Bt.b.cyc, st));
    return TVS_OK;
}

}  // namespace

extern "C" {

int tvs_iterate_batch(tvs_ctx *ctx, const tvs_params *p, int32_t S, int32_t K, void *stream)
{
    if (!ctx) return TVS_EINVAL;
    ctx->err.clear();
    if (S < 1 || S > 32) return fail(ctx, TVS_EINVAL, "batch size must lie in [1, 32]");
    if (!p) return fail(ctx, TVS_EINVAL, "params is NULL");
    if (K < 0) return fail(ctx, TVS_EINVAL, "K must be >= 0");
    for (int q = 0; q < S; q++) {
        int rc = validate_params(ctx, p + q);
        if (rc) return rc;
        if (p[q].variant == TVS_OTVS || (p[q].variant == TVS_NTVS && p[q].tv_check))
            return fail(ctx, TVS_EINVAL, "batches take unchecked schedules only");
    }
    if (!ctx->loaded) return fail(ctx, TVS_ESTATE, "tvs_iterate_batch before tvs_load_histories");
    HIPCHK(hipSetDevice(ctx->cfg.device));
    hipStream_t st = pick(ctx, stream);
    // the chunk buffers must be free of the single-image sweep's work (its
    // last reads are marked by the buffer-free events, also when it ran on
    // another stream)
    HIPCHK(hipStreamSynchronize(ctx->fill_stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctx->cfg.path_mode == TVS_PATH_ON_THE_FLY)
        for (int q = 0; q < kChunkBuffers; q++) HIPCHK(hipStreamWaitEvent(st, ctx->ev_free[q], 0));
    auto &B = ctx->batch;
    bool same = B.valid && B.S == S;
    for (int q = 0; same && q < S; q++) same = same_params(B.p[q], p[q]);
    if (!same) {
        int rc = batch_init(ctx, p, S, st);
        if (rc) return rc;
    }
    B.ms_total = 0;
    B.cycles = 0;
    if (K == 0) return TVS_OK;

    // beta of every (cycle, step, setting) of this call, drawn on the host
    int nmax = 0;
    for (int q = 0; q < S; q++) nmax = std::max(nmax, (int)p[q].N);
    const int64_t need = std::max<int64_t>((int64_t)K * std::max(nmax, 1) * S, 1);
    if (need > B.beta_cap) {
        dfree(ctx, &B.b.beta_tab, (size_t)B.beta_cap);
        B.beta_cap = 0;
        int rc = dalloc(ctx, &B.b.beta_tab, (size_t)need);
        if (rc) return rc;
        B.beta_cap = need;
    }
    std::vector<double> beta((size_t)need, 0.0);
    for (int32_t kk = 0; kk < K; kk++) {
        const int64_t k = B.k + kk;
        for (int q = 0; q < S; q++) {
            if (p[q].variant == TVS_NTVS) B.ell[q] = draw_ell(k, B.ell[q], B.rng[q]);
            for (int n = 0; n < p[q].N; n++) {
                double b = (p[q].variant == TVS_DECOUPLED)
                               ? std::pow(p[q].alpha, (double)(n + 1)) * std::pow(p[q].gamma, (double)k)
                               : std::pow(p[q].alpha, (double)B.ell[q]);
                beta[((size_t)kk * nmax + n) * S + q] = b;
                B.ell[q] += 1;
            }
        }
    }
    B.k += K;
    HIPCHK(hipMemcpyAsync(B.b.beta_tab, beta.data(), sizeof(double) * need, hipMemcpyHostToDevice, st));
    HIPCHK(tvs::launch_set_counter(B.b.cyc, 0, st));

    // capture one cycle, replay it K times
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
    int rc = batch_cycle(ctx, nmax, st);
    hipError_t ce = hipStreamEndCapture(st, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ce != hipSuccess) return fail(ctx, TVS_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
    ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ce != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(ctx, TVS_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ce));
    }
    ctx->tev_used = 0;
    ctx->spans.clear();
    ctx->timed = false;
    std::vector<long> ev;
    ev.push_back(mark(ctx, st));
    for (int32_t kk = 0; kk < K && ce == hipSuccess; kk++) {
        ce = hipGraphLaunch(exec, st);
        ev.push_back(mark(ctx, st));
    }
    hipError_t se = hipStreamSynchronize(st);
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (ce != hipSuccess) return fail(ctx, TVS_EDEVICE, std::string("graph launch: ") + hipGetErrorString(ce));
    if (se != hipSuccess) return fail(ctx, TVS_EDEVICE, std::string("batch sync: ") + hipGetErrorString(se));
    for (size_t q = 1; q < ev.size(); q++) {
        float ms = 0;
        if (ev[q - 1] >= 0 && ev[q] >= 0 &&
            hipEventElapsedTime(&ms, ctx->tev[(size_t)ev[q - 1]], ctx->tev[(size_t)ev[q]]) == hipSuccess)
            B.ms_total += ms;
    }
    B.cycles = K;
    ctx->tev_used = 0;
    return TVS_OK;
}

int tvs_get_batch_image(tvs_ctx *ctx, int32_t s, float *out, int on_device, void *stream)
{
    if (!ctx) return TVS_EINVAL;
    ctx->err.clear();
    if (!out) return fail(ctx, TVS_EINVAL, "output is NULL");
    if (!ctx->batch.valid) return fail(ctx, TVS_ESTATE, "no batch");
    if (s < 0 || s >= ctx->batch.S) return fail(ctx, TVS_ERANGE, "setting outside the batch");
    HIPCHK(hipSetDevice(ctx->cfg.device));
    hipStream_t st = pick(ctx, stream);
    int rc = check_flags(ctx, st);
    if (rc) return rc;
    HIPCHK(tvs::launch_extract(ctx->gd, ctx->batch.b, s, ctx->xio, st));
    HIPCHK(hipMemcpyAsync(out, ctx->xio, sizeof(float) * ctx->nimg,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    if (!on_device) HIPCHK(hipStreamSynchronize(st));
    return TVS_OK;
}

extern "C++" {

// Launch-shape cache of the tuners: one line per measurement, "key values",
// the key a whitespace-free description of the device, grid, history count,
// B and path mode (plus the tuner's own tag); the last matching line wins.
static std::string tune_key(const tvs_ctx *ctx, const hipDeviceProp_t &prop, const char *tag)
{
    char key[512];
    std::snprintf(key, sizeof(key), "%s|%dx%dx%d|%.6gx%.6gx%.6g|H%lld|B%d|P%d%s", prop.gcnArchName,
                  ctx->grid.nx, ctx->grid.ny, ctx->grid.nz, ctx->grid.vx, ctx->grid.vy,
                  ctx->grid.vz, (long long)ctx->nh, ctx->cfg.block_size, ctx->cfg.path_mode, tag);
    return key;
}

// Calls fn(values) for every line of the cache file whose key is `key`.
template <typename F>
static void cache_scan(const char *path, const std::string &key, F fn)
{
    FILE *f = path ? std::fopen(path, "r") : nullptr;
    if (!f) return;
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
        char k[512];
        int used = 0;
        if (std::sscanf(line, "%511s%n", k, &used) == 1 && key == k) fn(line + used);
    }
    std::fclose(f);
}

static void cache_append(const char *path, const std::string &key, const std::string &values)
{
    if (!path) return;
    if (FILE *f = std::fopen(path, "a")) {
        std::fprintf(f, "%s %s\n", key.c_str(), values.c_str());
        std::fclose(f);
    }
}

}  // extern "C++"

int tvs_autotune(tvs_ctx *ctx, double lambda, const char *cache_path, tvs_tune_result *out,
                 void *stream)
{
    if (!ctx || !out) return TVS_EINVAL;
    ctx->err.clear();
    std::memset(out, 0, sizeof(*out));
    if (!finite_pos(lambda)) return fail(ctx, TVS_EINVAL, "lambda must be finite and > 0");
    if (!ctx->loaded) return fail(ctx, TVS_ESTATE, "tvs_autotune before tvs_load_histories");
    HIPCHK(hipSetDevice(ctx->cfg.device));
    hipStream_t st = pick(ctx, stream);
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, ctx->cfg.device));
    const std::string key = tune_key(ctx, prop, "");
    if (cache_path) {
        cache_scan(cache_path, key, [&](const char *v) {
            int th = 0, sw = 0, pct = -1;
            double ms = 0;
            const int got = std::sscanf(v, "%d %d %lf %d", &th, &sw, &ms, &pct);
            if (got >= 3 && (th == 64 || th == 128 || th == 256) && (sw == 1 || sw == 2)) {
                out->tile_threads = th;
                out->sweep_kernel = sw;
                out->ms_per_block = ms;
                out->fill_wide_pct = (got == 4 && pct >= 0 && pct <= 100) ? pct
                                                                           : ctx->fill_wide_pct;
                out->from_cache = 1;
            }
        });
        if (out->from_cache) {
            ctx->threads = out->tile_threads;
            ctx->split = out->sweep_kernel == 2 ? 1 : 0;
            ctx->fill_wide_pct = out->fill_wide_pct;
            return TVS_OK;
        }
    }
    const int64_t B = ctx->cfg.block_size;
    // enough blocks that the candidates' differences stand above the spread
    // of a step's duration (48 blocks picked 64-lane tiles for the 256x256x32
    // fixed-point store, 20 % slower per whole sweep than 128)
    const int64_t nb = std::min<int64_t>(ctx->nblocks, 1024);
    out->fill_wide_pct = ctx->fill_wide_pct;
    if (nb == 0) {
        out->tile_threads = ctx->threads;
        out->sweep_kernel = ctx->split ? 2 : 1;
        return TVS_OK;
    }
    HIPCHK(hipStreamSynchronize(ctx->fill_stream));
    double *saved = nullptr;
    int rc = dalloc(ctx, &saved, (size_t)ctx->nvox);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(saved, ctx->x, sizeof(double) * ctx->nvox, hipMemcpyDeviceToDevice, st));
    const int ths[3] = {64, 128, 256};
    const int old_threads = ctx->threads, old_split = ctx->split;
    double best = 1e300;
    int nc = 0;
    for (int sw = 1; sw <= 2 && rc == TVS_OK; sw++) {
        for (int ti = 0; ti < 3 && rc == TVS_OK; ti++) {
            ctx->threads = ths[ti];
            ctx->split = sw == 2 ? 1 : 0;
            double tbest = 1e300;
            for (int rep = 0; rep < 3 && rc == TVS_OK; rep++) {
                ctx->tev_used = 0;
                ctx->spans.clear();
                long a = mark(ctx, st);
                rc = run_sweep(ctx, lambda, st, std::min(nb * B, ctx->nh));
                long b = mark(ctx, st);
                if (rc) break;
                hipError_t e = hipMemcpyAsync(ctx->x, saved, sizeof(double) * ctx->nvox,
                                              hipMemcpyDeviceToDevice, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                if (e == hipSuccess) e = hipStreamSynchronize(ctx->fill_stream);
                float ms = 0;
                if (e == hipSuccess && a >= 0 && b >= 0)
                    e = hipEventElapsedTime(&ms, ctx->tev[(size_t)a], ctx->tev[(size_t)b]);
                if (e != hipSuccess) {
                    rc = fail(ctx, TVS_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
                    break;
                }
                if (rep > 0) tbest = std::min(tbest, (double)ms / nb);   // rep 0 warms up
            }
            if (rc) break;
            if (nc < 8) {
                out->cand_threads[nc] = ths[ti];
                out->cand_sweep[nc] = sw;
                out->cand_ms[nc] = tbest;
                nc++;
            }
            if (tbest < best) {
                best = tbest;
                out->tile_threads = ths[ti];
                out->sweep_kernel = sw;
                out->ms_per_block = tbest;
            }
        }
    }
    out->n_candidates = nc;
    if (rc || best == 1e300) {
        dfree(ctx, &saved, (size_t)ctx->nvox);
        ctx->tev_used = 0;
        ctx->spans.clear();
        ctx->timed = false;
        ctx->threads = old_threads;
        ctx->split = old_split;
        return rc ? rc : fail(ctx, TVS_EDEVICE, "autotune: no candidate ran");
    }
    ctx->threads = out->tile_threads;
    ctx->split = out->sweep_kernel == 2 ? 1 : 0;
    // on the fly: whole sweeps (the row formation beside the chain) for the
    // share of chunks formed at the row kernel's full occupancy; with one
    // chunk the share does not matter
    const int64_t nchunks = (ctx->nh + ctx->chunk - 1) / ctx->chunk;
    if (ctx->cfg.path_mode == TVS_PATH_ON_THE_FLY && nchunks > 1) {
        const int pcts[6] = {0, 20, 40, 60, 80, 100};
        const int old_pct = ctx->fill_wide_pct;
        double pbest = 1e300;
        for (int pi = 0; pi < 6 && rc == TVS_OK; pi++) {
            ctx->fill_wide_pct = pcts[pi];
            ctx->tev_used = 0;
            ctx->spans.clear();
            long a = mark(ctx, st);
            rc = run_sweep(ctx, lambda, st);
            long b = mark(ctx, st);
            if (rc) break;
            hipError_t e = hipMemcpyAsync(ctx->x, saved, sizeof(double) * ctx->nvox,
                                          hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->fill_stream);
            float ms = 0;
            if (e == hipSuccess && a >= 0 && b >= 0)
                e = hipEventElapsedTime(&ms, ctx->tev[(size_t)a], ctx->tev[(size_t)b]);
            if (e != hipSuccess) {
                rc = fail(ctx, TVS_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
                break;
            }
            out->cand_pct[out->n_fill] = pcts[pi];
            out->cand_sweep_ms[out->n_fill] = ms;
            out->n_fill++;
            if (ms < pbest) {
                pbest = ms;
                out->fill_wide_pct = pcts[pi];
            }
        }
        ctx->fill_wide_pct = rc ? old_pct : out->fill_wide_pct;
    }
    dfree(ctx, &saved, (size_t)ctx->nvox);
    ctx->tev_used = 0;
    ctx->spans.clear();
    ctx->timed = false;
    if (rc) return rc;
    char vals[128];
    std::snprintf(vals, sizeof(vals), "%d %d %.6f %d", out->tile_threads, out->sweep_kernel,
                  out->ms_per_block, out->fill_wide_pct);
    cache_append(cache_path, key, vals);
    return TVS_OK;
}

int tvs_autotune_batch(tvs_ctx *ctx, const tvs_params *p, int32_t S, const char *cache_path,
                       tvs_batch_tune_result *out, void *stream)
{
    if (!ctx || !out) return TVS_EINVAL;
    ctx->err.clear();
    std::memset(out, 0, sizeof(*out));
    if (S < 1 || S > 32) return fail(ctx, TVS_EINVAL, "batch size must lie in [1, 32]");
    if (!p) return fail(ctx, TVS_EINVAL, "params is NULL");
    for (int q = 0; q < S; q++) {
        int rc = validate_params(ctx, p + q);
        if (rc) return rc;
    }
    if (!ctx->loaded) return fail(ctx, TVS_ESTATE, "tvs_autotune_batch before tvs_load_histories");
    HIPCHK(hipSetDevice(ctx->cfg.device));
    hipStream_t st = pick(ctx, stream);
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, ctx->cfg.device));
    const std::string key = tune_key(ctx, prop, ("|S" + std::to_string(S)).c_str());
    if (cache_path) {
        cache_scan(cache_path, key, [&](const char *v) {
            int th = 0, gp = 0;
            double ms = 0;
            if (std::sscanf(v, "%d %d %lf", &th, &gp, &ms) == 3 && tvs::batch_shape_ok(th, gp)) {
                out->threads = th;
                out->group = gp;
                out->ms_per_block = ms;
                out->from_cache = 1;
            }
        });
        if (out->from_cache) {
            ctx->bthreads = out->threads;
            ctx->bgroup = out->group;
            return TVS_OK;
        }
    }
    const int64_t B = ctx->cfg.block_size;
    const bool otf = ctx->cfg.path_mode == TVS_PATH_ON_THE_FLY;
    // the first blocks of the first chunk (formed here on the fly)
    int64_t nb = std::min<int64_t>(ctx->nblocks, 48);
    if (otf) nb = std::min<int64_t>(nb, ctx->chunk / B);
    if (nb == 0) {
        out->threads = ctx->bthreads;
        out->group = ctx->bgroup;
        return TVS_OK;
    }
    HIPCHK(hipStreamSynchronize(ctx->fill_stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    int rc = batch_init(ctx, p, S, st);
    if (rc) return rc;
    auto &Bt = ctx->batch;
    if (otf) {
        for (int q = 0; q < kChunkBuffers; q++) HIPCHK(hipStreamWaitEvent(st, ctx->ev_free[q], 0));
        tvs::TileFill f = chunk_fill(ctx, 0, std::min(ctx->chunk, ctx->nh));
        f.max_wgs = 0;
        HIPCHK(tvs::launch_rows_fill_tiled(ctx->gd, hist_dev(ctx), ctx->mlp, f, st));
        HIPCHK(hipEventRecord(ctx->ev_free[chunk_buffer(ctx, 0)], st));
    }
    const int ths[2] = {128, 256}, gps[4] = {2, 4, 8, 16};
    const int old_t = ctx->bthreads, old_g = ctx->bgroup;
    double best = 1e300;
    int nc = 0;
    for (int ti = 0; ti < 2 && rc == TVS_OK; ti++) {
        for (int gi = 0; gi < 4 && rc == TVS_OK; gi++) {
            ctx->bthreads = ths[ti];
            ctx->bgroup = gps[gi];
            double tbest = 1e300;
            for (int rep = 0; rep < 3 && rc == TVS_OK; rep++) {
                ctx->tev_used = 0;
                ctx->spans.clear();
                hipError_t e = tvs::launch_zero_i64(Bt.dot, 3 * B * S, st);
                long a = mark(ctx, st);
                for (int64_t b = 0; b <= nb && e == hipSuccess; b++) {
                    tvs::DropTileArgs A;
                    if (b > 0) A.P = block_view(ctx, b - 1, Bt.dot, B * S);
                    if (b < nb) A.C = block_view(ctx, b, Bt.dot, B * S);
                    A.x = Bt.b.x;
                    A.big = ctx->big;
                    A.dot_max = ctx->dot_max;
                    A.zero = Bt.dot + ((b + 1) % 3) * B * S;
                    A.B = B;
                    A.err = ctx->flags + kFlagRange;
                    A.tiles = ctx->act;
                    A.nact = ctx->nact;
                    e = tvs::launch_drop_tiles_batch(A, Bt.b, ctx->ntiles, ctx->bthreads,
                                                     ctx->bgroup, st);
                }
                long bm = mark(ctx, st);
                if (e == hipSuccess) e = hipStreamSynchronize(st);
                float ms = 0;
                if (e == hipSuccess && a >= 0 && bm >= 0)
                    e = hipEventElapsedTime(&ms, ctx->tev[(size_t)a], ctx->tev[(size_t)bm]);
                if (e != hipSuccess) {
                    rc = fail(ctx, TVS_EDEVICE, std::string("batch autotune: ") + hipGetErrorString(e));
                    break;
                }
                if (rep > 0) tbest = std::min(tbest, (double)ms / (double)nb);   // rep 0 warms up
            }
            if (rc) break;
            if (nc < 8) {
                out->cand_threads[nc] = ths[ti];
                out->cand_group[nc] = gps[gi];
                out->cand_ms[nc] = tbest;
                nc++;
            }
            if (tbest < best) {
                best = tbest;
                out->threads = ths[ti];
                out->group = gps[gi];
                out->ms_per_block = tbest;
            }
        }
    }
    ctx->tev_used = 0;
    ctx->spans.clear();
    ctx->timed = false;
    out->n_candidates = nc;
    // the timed steps moved the batch images: the next batch starts afresh
    Bt.valid = false;
    if (rc || best == 1e300) {
        ctx->bthreads = old_t;
        ctx->bgroup = old_g;
        return rc ? rc : fail(ctx, TVS_EDEVICE, "batch autotune: no candidate ran");
    }
    ctx->bthreads = out->threads;
    ctx->bgroup = out->group;
    rc = check_flags(ctx, st);
    if (rc) return rc;
    char vals[96];
    std::snprintf(vals, sizeof(vals), "%d %d %.6f", out->threads, out->group, out->ms_per_block);
    cache_append(cache_path, key, vals);
    return TVS_OK;
}

}  // extern "C"
