// C ABI of libsymba: context, argument checks, task planning and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/symba.h"
#include "symba_arena.h"
#include "symba_internal.h"

using symba::Desc;

struct symba_ctx {
    int device = 0;
    int64_t max_n = 0;
    int64_t max_pairs = 0;
    int max_problems = 0;
    // scratch
    int32_t *parent = nullptr;   // [max_n] union-find offsets, zero between calls
    int32_t *touched = nullptr;  // [max_n]
    int32_t *blk_groups = nullptr;  // [max_n / kFinBodies + max_problems] groups per final-kernel body block
    double *mom = nullptr;          // [2][mom_blocks][3] momentum partial sums of symba_step(_batch)
    int64_t mom_blocks = 0;         // step_blocks(max_n) + max_problems
    symba::StepDesc *steps_dev = nullptr;     // [max_problems] drift descriptors of a step batch
    symba::StepDesc *steps_pinned = nullptr;
    hipEvent_t steps_done = nullptr;
    bool steps_pending = false;
    int2 *pairs = nullptr;       // [max_pairs]
    int4 *sorted = nullptr;      // [max_pairs]
    int32_t *bcnt = nullptr;     // [max_n]
    int32_t *bfill = nullptr;    // [max_n]
    unsigned long long *ctr = nullptr;  // [kCtrSlots * max_problems]
    unsigned long long *stats = nullptr;  // [kStatSlots]
    int32_t *bin_key = nullptr, *bin_tmp = nullptr, *bin_idx = nullptr;  // [max_n] each
    double *binned = nullptr;    // [8 * max_n]
    double *tbox = nullptr;      // [max_boxes * kBoxDoubles]
    int64_t max_boxes = 0;
    unsigned long long *bin_bbox = nullptr;  // [12], zero between calls
    int32_t *bin_temp = nullptr;             // [kBinTempInts]: cell counts and fills (zero between calls), starts
    double *partial = nullptr;
    size_t partial_bytes = 0;
    bool partial_captured = false;          // a captured call references the current partial buffer
    std::vector<double *> partial_retired;  // earlier partial buffers a captured call may use (freed at destroy)
    // capture arena: descriptors of calls made under stream capture, append-only
    char *cap_pinned = nullptr;
    char *cap_dev = nullptr;
    symba::BumpArena cap_arena;
    Desc *descs_dev = nullptr;   // [max_problems]
    Desc *descs_pinned = nullptr;
    std::vector<Desc> descs_last;  // what descs_dev currently holds
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;
    // options
    int opt_rows = 0, opt_field_rows = 0, opt_screen = 0, opt_timing = 0, opt_bin = 0, opt_acc = 0;
    int opt_split = -1;  // split diagonals of the folded triangle, -1 = automatic
    int opt_enc_fuse = 1;  // fused encounter-step launches for one-block problems
    int opt_enc_regs = 1;  // small encounter groups integrated in registers
    double *ind = nullptr;  // [max_n / kIndBodies + max_problems][3] indirect-term partial sums (SYMBA_ACC_HELIO)
    // tile rows chosen by symba_autotune per size class (floor(log2(n_tri))), 0 = not tuned
    int tuned_rows[64] = {};
    // split diagonals + 1 chosen with those rows by symba_autotune, 0 = not tuned
    int tuned_split[64] = {};
    // timing events (SYMBA_OPT_TIMING): three per timed call
    std::vector<hipEvent_t> events;
    size_t timed_calls = 0;
    // encounter step (symba_step_enc): group table and flags
    int32_t *enc_gp = nullptr;      // [kEncMaxPairs]
    int32_t *enc_gstart = nullptr;  // [kEncMaxPairs + 1]
    int32_t *enc_gskip = nullptr;   // [kEncMaxPairs]
    int32_t *enc_ctl = nullptr;     // [kEncCtlInts], zero between calls
    int32_t *ingroup = nullptr;     // [max_n], zero between calls
    // the scratch is a fixed region (symba_kick_encounter_noalloc): nothing
    // may be allocated, a call that would need more returns SYMBA_ETOOBIG
    bool fixed_scratch = false;
};

namespace {

constexpr int kMaxProblems = 4096;
constexpr size_t kCaptureArenaBytes = size_t(8) << 20;  // descriptors of captured calls
constexpr int kMaxSplit = 8;  // most split diagonals SYMBA_OPT_SPLIT accepts
// Pair-scatter blocks (final kernel) and closing blocks per problem: a single
// call spreads them wide, a batch of many problems less so.
constexpr int kScatterBlocks = 16, kCloseBlocks = 32;
constexpr int kScatterBlocksBatch = 2, kCloseBlocksBatch = 2;
constexpr size_t kMaxTimedCalls = 4096;

// Events for the next timed call, or null when timing is off or the pool is full.
hipEvent_t *timing_slot(symba_ctx *c) {
    if (!c->opt_timing || c->timed_calls >= kMaxTimedCalls) return nullptr;
    const size_t need = 3 * (c->timed_calls + 1);
    while (c->events.size() < need) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->events.push_back(e);
    }
    hipEvent_t *ev = c->events.data() + 3 * c->timed_calls;
    ++c->timed_calls;
    return ev;
}

// Bodies per lane of the triangle tiles: R = 1 keeps small problems spread
// over many workgroups; larger R amortises the lane rotation and shrinks the
// partial-sum buffer (B x 3 x N doubles, B = N / (64 R)).  A forced option
// wins, then a size class tuned by symba_autotune, then the built-in table.
int size_class(int64_t n_tri) {
    int c = 0;
    while (c < 63 && (int64_t(2) << c) <= n_tri) ++c;
    return c;
}

int rows_for(const symba_ctx *c, int64_t n_tri) {
    if (c->opt_rows) return c->opt_rows;
    if (n_tri > 0 && c->tuned_rows[size_class(n_tri)]) return c->tuned_rows[size_class(n_tri)];
    if (n_tri >= 30000) return 4;
    if (n_tri >= 4000) return 2;
    return 1;
}

int field_rows_for(int64_t n_field, int opt) {
    if (opt) return opt;
    return n_field >= 200000 ? 2 : 1;
}

// Split diagonals of the folded triangle (tile pairs launched last to even
// out the end of the tile kernel).  A tuning knob.
#ifndef SYMBA_TAIL_SPLIT
#define SYMBA_TAIL_SPLIT 2
#endif

// The split only pays when the launch is a few rounds of workgroups deep, so
// that its ragged end is a sizeable part of the kernel; deeper launches keep
// every block pair whole.  Rounds are counted against MI355X's 256 CUs at the
// tile kernel's occupancy (6, 4, 2 workgroups per CU for 1, 2, 4 rows): a
// fixed planning constant, so that the plan, and with it the summation order,
// does not depend on the device.
constexpr int64_t kPlanCUs = 256;
constexpr int64_t kSplitMaxRounds = 6;

int64_t tail_split(int64_t B, int rows) {
    const int64_t slots = kPlanCUs * (rows == 1 ? 6 : rows == 2 ? 4 : 2);
    if (symba::fold_count(B) >= kSplitMaxRounds * slots) return 0;
    return symba::split_diagonals(B, rows, SYMBA_TAIL_SPLIT);
}

// Split diagonals wanted for a problem of n_tri massive bodies run with
// `rows`: SYMBA_OPT_SPLIT when set, else what symba_autotune chose for the
// size class together with these rows, else -1 (the rule of tail_split).
int split_for(const symba_ctx *c, int64_t n_tri, int rows) {
    if (c->opt_split >= 0) return c->opt_split;
    if (n_tri > 0) {
        const int k = size_class(n_tri);
        if (c->tuned_split[k] && c->tuned_rows[k] == rows) return c->tuned_split[k] - 1;
    }
    return -1;
}

struct Plan {
    int64_t n_rows, n_tri, B, n_split, n_whole, n_slots, n_tri_tasks, n_field_tasks, n_blk;
    int64_t n_fblocks, n_fslots;  // field blocks; segments of the massive rows per field block
    int rows;
    size_t partial_doubles;
};

// split: split diagonals wanted (clamped to what the fold allows), -1 for
// the rule of tail_split.
Plan make_plan(int64_t n, int64_t n_m, int rows, int field_rows, int split) {
    Plan p{};
    p.n_rows = std::min(n_m, n - 1);
    p.n_tri = n_m >= n - 1 ? n : n_m;
    const int64_t S = (int64_t)rows * symba::kWave;
    const int64_t F = (int64_t)field_rows * symba::kWave;
    p.rows = rows;
    if (p.n_rows > 0) {
        p.B = (p.n_tri + S - 1) / S;
        p.n_split = split < 0 ? tail_split(p.B, rows) : symba::split_diagonals(p.B, rows, split);
        p.n_whole = symba::whole_count(p.B, p.n_split);
        p.n_tri_tasks = p.n_whole + p.n_split * p.B * rows * rows;
        p.n_slots = symba::partial_slots(p.B, rows, p.n_split);
        p.n_fblocks = (n - p.n_tri + F - 1) / F;
        p.n_fslots = p.n_fblocks > 0 ? (p.n_rows + symba::kFieldSegRows - 1) / symba::kFieldSegRows : 0;
        p.n_field_tasks = p.n_fblocks * p.n_fslots;
    }
    p.n_blk = (n + symba::kFinBodies - 1) / symba::kFinBodies;
    p.partial_doubles = (size_t)p.n_slots * 3 * (size_t)p.n_tri + (size_t)p.n_fslots * 3 * (size_t)(n - p.n_tri);
    return p;
}

// Problems with at least this many massive bodies are binned by default (the
// screen-free tiles then repay the two binning launches).
constexpr int64_t kBinMinTri = 20000;

bool use_bin(const symba_ctx *c, int64_t n, int64_t n_m) {
    const int64_t n_tri = n_m >= n - 1 ? n : n_m;
    if (std::min(n_m, n - 1) < 1 || c->opt_bin == 1) return false;
    return c->opt_bin == 2 || n_tri >= kBinMinTri;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// The FP32 screen unless the FP64 one is asked for: on gfx950 it issues one
// more operation per pair but reads half the LDS bytes per streamed body and
// holds fewer registers, and measures slightly faster.
int screen32(const symba_ctx *c) { return c->opt_screen == SYMBA_SCREEN_FP64 ? 0 : 1; }

// Points the descriptor's tile-kernel inputs at the binned copies (scratch at
// body offset body_off, tile boxes at box_off) or at the caller's inputs.
// Returns 1 when the problem is binned.  The binning temporaries are shared:
// the problems of a call are binned one after the other.
int wire_binning(const symba_ctx *c, Desc &d, bool bin, int64_t body_off, int64_t box_off) {
    d.bx = d.x; d.by = d.y; d.bz = d.z; d.bm = d.m; d.bvx = d.vx; d.bvy = d.vy; d.bvz = d.vz; d.brh = d.rh;
    d.bidx = nullptr;
    d.tbox = nullptr;
    d.bin_key = d.bin_tmp = d.bin_idx = nullptr;
    d.binned = d.tbox_w = nullptr;
    d.bin_bbox = nullptr;
    d.bin_hist = d.bin_fill = d.bin_start = nullptr;
    d.n_tboxes = d.n_boxes = 0;
    if (!bin) return 0;
    const int64_t n = d.n;
    d.bin_key = c->bin_key + body_off;
    d.bin_tmp = c->bin_tmp + body_off;
    d.bin_idx = c->bin_idx + body_off;
    d.binned = c->binned + 8 * body_off;
    d.tbox_w = c->tbox + symba::kBoxDoubles * box_off;
    d.bx = d.binned; d.by = d.binned + n; d.bz = d.binned + 2 * n; d.bm = d.binned + 3 * n;
    d.bvx = d.binned + 4 * n; d.bvy = d.binned + 5 * n; d.bvz = d.binned + 6 * n; d.brh = d.binned + 7 * n;
    d.bidx = d.bin_idx;
    d.tbox = d.tbox_w;
    d.n_tboxes = ceil_div(d.n_tri, symba::kWave);
    d.n_boxes = d.n_tboxes + ceil_div(n - d.n_tri, symba::kWave);
    d.bin_bbox = c->bin_bbox;
    d.bin_hist = c->bin_temp;
    d.bin_fill = c->bin_temp + 2 * 2048;
    d.bin_start = c->bin_temp + 4 * 2048;
    return 1;
}

bool bad_scalar(double dt, double f) { return !(dt >= 0.0) || !std::isfinite(dt) || !(f > 0.0) || !std::isfinite(f); }

bool bad_state(const symba_state *s) {
    return !s || !s->x || !s->y || !s->z || !s->vx || !s->vy || !s->vz || !s->m || !s->rh;
}

bool bad_out(const symba_out *o) {
    return !o || !o->ax || !o->ay || !o->az || !o->n_pairs || !o->group_id || !o->n_groups ||
           !o->status || o->pair_cap < 0 || (o->pair_cap > 0 && (!o->pair_i || !o->pair_j));
}

// True while `stream` is being captured into a graph (nothing may be
// allocated, freed or synchronised then).
bool is_capturing(hipStream_t stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

// The partial-sum buffer for a call that needs `doubles` of it (see
// symba::plan_partial): grown geometrically when too small; a buffer a
// captured call has used is retired rather than freed; no growth under
// capture (SYMBA_EINVAL: run the shape once outside capture first).
int grow_partial(symba_ctx *c, size_t doubles, bool capturing) {
    const size_t need = std::max<size_t>(doubles * sizeof(double), 256);
    if (c->fixed_scratch) return need <= c->partial_bytes ? SYMBA_OK : SYMBA_ETOOBIG;
    const symba::PartialAction a = symba::plan_partial(c->partial_bytes, need, c->partial_captured, capturing);
    if (a.kind == symba::PartialAction::Refuse) return SYMBA_EINVAL;
    if (a.kind == symba::PartialAction::Grow) {
        double *fresh = nullptr;
        if (hipMalloc(&fresh, a.new_bytes) != hipSuccess) return SYMBA_ENOMEM;
        if (c->partial) {
            if (a.retire_old)
                c->partial_retired.push_back(c->partial);
            else if (hipFree(c->partial) != hipSuccess)
                return SYMBA_EDEVICE;
        }
        c->partial = fresh;
        c->partial_bytes = a.new_bytes;
        c->partial_captured = false;
    }
    if (capturing) c->partial_captured = true;
    return SYMBA_OK;
}

// Device copy of `bytes` of host data for a call made under capture: staged
// in the capture arena (pinned and device halves at the same offset), copied
// by a captured node that every replay repeats from the same, never
// rewritten, pinned bytes.  Null when the arena is full.
void *capture_upload(symba_ctx *c, const void *src, size_t bytes, hipStream_t stream) {
    size_t off = 0;
    if (!c->cap_arena.alloc(bytes, 256, off)) return nullptr;
    std::memcpy(c->cap_pinned + off, src, bytes);
    if (hipMemcpyAsync(c->cap_dev + off, c->cap_pinned + off, bytes, hipMemcpyHostToDevice, stream) != hipSuccess)
        return nullptr;
    return c->cap_dev + off;
}

void fill_desc(Desc &d, const symba_state &s, const symba_out &o, int64_t n, int64_t n_m, double dt,
               double f, const Plan &p, int field_rows) {
    std::memset(&d, 0, sizeof d);
    d.x = s.x; d.y = s.y; d.z = s.z; d.vx = s.vx; d.vy = s.vy; d.vz = s.vz; d.m = s.m; d.rh = s.rh;
    d.ax = o.ax; d.ay = o.ay; d.az = o.az;
    d.pair_i = o.pair_i; d.pair_j = o.pair_j; d.pair_cap = o.pair_cap;
    d.n_pairs_out = o.n_pairs; d.group_id = o.group_id; d.n_groups_out = o.n_groups; d.status_out = o.status;
    d.n = n; d.n_rows = p.n_rows; d.n_tri = p.n_tri; d.dt = dt; d.f = f;
    d.k15 = 1.5; d.k1875 = 1.875;
    d.screen_dt2 = 2.0 * (1.0 + 0x1p-20) * (dt * dt);
    d.B = p.B; d.n_split = p.n_split; d.n_whole = p.n_whole; d.n_slots = p.n_slots;
    d.n_tri_tasks = p.n_tri_tasks; d.n_tasks = p.n_tri_tasks + p.n_field_tasks;
    d.n_blk = p.n_blk; d.field_block = (int64_t)field_rows * symba::kWave;
    d.n_fslots = p.n_fslots;
    d.n_fblocks = p.n_fblocks;
    (void)n_m;
}

}  // namespace

extern "C" {

const char *symba_strerror(int code) {
    switch (code) {
        case SYMBA_OK: return "ok";
        case SYMBA_EINVAL: return "invalid argument";
        case SYMBA_ENOMEM: return "device allocation failed";
        case SYMBA_EDEVICE: return "HIP runtime error";
        case SYMBA_ETOOBIG: return "problem larger than the context was created for";
        default: return "unknown error";
    }
}

int symba_ctx_create(symba_ctx **out, int device, int64_t max_n, int64_t max_pairs, uint32_t flags) {
    if (!out) return SYMBA_EINVAL;
    *out = nullptr;
    if (max_n < 1 || max_pairs < 0 || flags != 0 || max_n > INT32_MAX) return SYMBA_EINVAL;
    if (max_pairs == 0) max_pairs = std::max<int64_t>(4 * max_n, 4096);
    if (max_pairs > INT32_MAX) return SYMBA_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return SYMBA_EDEVICE;
    symba_ctx *c = new (std::nothrow) symba_ctx();
    if (!c) return SYMBA_ENOMEM;
    c->device = device;
    c->max_n = max_n;
    c->max_pairs = max_pairs;
    c->max_problems = kMaxProblems;
    c->max_boxes = max_n / symba::kWave + 2 * (int64_t)kMaxProblems;
    c->mom_blocks = symba::step_blocks(max_n) + kMaxProblems;
    bool ok = hipMalloc(&c->parent, sizeof(int32_t) * max_n) == hipSuccess &&
              hipMalloc(&c->touched, sizeof(int32_t) * max_n) == hipSuccess &&
              hipMalloc(&c->blk_groups, sizeof(int32_t) * (max_n / symba::kFinBodies + kMaxProblems)) ==
                  hipSuccess &&
              hipMalloc(&c->mom, sizeof(double) * 6 * (symba::step_blocks(max_n) + kMaxProblems)) == hipSuccess &&
              hipMalloc(&c->steps_dev, sizeof(symba::StepDesc) * kMaxProblems) == hipSuccess &&
              hipMalloc(&c->ind, sizeof(double) * 3 * (max_n / symba::kIndBodies + kMaxProblems)) == hipSuccess &&
              hipHostMalloc(&c->steps_pinned, sizeof(symba::StepDesc) * kMaxProblems, hipHostMallocDefault) ==
                  hipSuccess &&
              hipEventCreateWithFlags(&c->steps_done, hipEventDisableTiming) == hipSuccess &&
              hipMalloc(&c->pairs, sizeof(int2) * max_pairs) == hipSuccess &&
              hipMalloc(&c->sorted, sizeof(int4) * max_pairs) == hipSuccess &&
              hipMalloc(&c->bcnt, sizeof(int32_t) * max_n) == hipSuccess &&
              hipMalloc(&c->bfill, sizeof(int32_t) * max_n) == hipSuccess &&
              hipMalloc(&c->ctr, sizeof(unsigned long long) * symba::kCtrSlots * kMaxProblems) == hipSuccess &&
              hipMalloc(&c->stats, sizeof(unsigned long long) * symba::kStatSlots) == hipSuccess &&
              hipMalloc(&c->bin_key, sizeof(int32_t) * max_n) == hipSuccess &&
              hipMalloc(&c->bin_tmp, sizeof(int32_t) * max_n) == hipSuccess &&
              hipMalloc(&c->bin_idx, sizeof(int32_t) * max_n) == hipSuccess &&
              hipMalloc(&c->binned, sizeof(double) * 8 * max_n) == hipSuccess &&
              hipMalloc(&c->tbox, sizeof(double) * symba::kBoxDoubles * c->max_boxes) == hipSuccess &&
              hipMalloc(&c->bin_bbox, sizeof(unsigned long long) * 12) == hipSuccess &&
              hipMalloc(&c->bin_temp, sizeof(int32_t) * symba::kBinTempInts) == hipSuccess &&
              hipMalloc(&c->descs_dev, sizeof(Desc) * kMaxProblems) == hipSuccess &&
              hipMalloc(&c->cap_dev, kCaptureArenaBytes) == hipSuccess &&
              hipHostMalloc(&c->cap_pinned, kCaptureArenaBytes, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc(&c->descs_pinned, sizeof(Desc) * kMaxProblems, hipHostMallocDefault) == hipSuccess &&
              hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming) == hipSuccess &&
              hipMalloc(&c->enc_gp, sizeof(int32_t) * symba::kEncMaxPairs) == hipSuccess &&
              hipMalloc(&c->enc_gstart, sizeof(int32_t) * (symba::kEncMaxPairs + 1)) == hipSuccess &&
              hipMalloc(&c->enc_gskip, sizeof(int32_t) * symba::kEncMaxPairs) == hipSuccess &&
              hipMalloc(&c->enc_ctl, sizeof(int32_t) * symba::kEncCtlInts) == hipSuccess &&
              hipMalloc(&c->ingroup, sizeof(int32_t) * max_n) == hipSuccess;
    c->cap_arena = symba::BumpArena(kCaptureArenaBytes);
    if (ok) {
        ok = hipMemset(c->parent, 0, sizeof(int32_t) * max_n) == hipSuccess &&
             hipMemset(c->touched, 0, sizeof(int32_t) * max_n) == hipSuccess &&
             hipMemset(c->bcnt, 0, sizeof(int32_t) * max_n) == hipSuccess &&
             hipMemset(c->bin_bbox, 0, sizeof(unsigned long long) * 12) == hipSuccess &&
             hipMemset(c->bin_temp, 0, sizeof(int32_t) * symba::kBinTempInts) == hipSuccess &&
             hipMemset(c->bfill, 0, sizeof(int32_t) * max_n) == hipSuccess &&
             hipMemset(c->ctr, 0, sizeof(unsigned long long) * symba::kCtrSlots * kMaxProblems) == hipSuccess &&
             hipMemset(c->stats, 0, sizeof(unsigned long long) * symba::kStatSlots) == hipSuccess &&
             hipMemset(c->enc_ctl, 0, sizeof(int32_t) * symba::kEncCtlInts) == hipSuccess &&
             hipMemset(c->ingroup, 0, sizeof(int32_t) * max_n) == hipSuccess &&
             hipDeviceSynchronize() == hipSuccess;
    }
    if (!ok) {
        symba_ctx_destroy(c);
        return SYMBA_ENOMEM;
    }
    *out = c;
    return SYMBA_OK;
}

int symba_ctx_destroy(symba_ctx *c) {
    if (!c) return SYMBA_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(c->parent);
    (void)hipFree(c->touched);
    (void)hipFree(c->blk_groups);
    (void)hipFree(c->mom);
    (void)hipFree(c->steps_dev);
    (void)hipFree(c->ind);
    if (c->steps_pinned) (void)hipHostFree(c->steps_pinned);
    if (c->steps_done) (void)hipEventDestroy(c->steps_done);
    (void)hipFree(c->pairs);
    (void)hipFree(c->sorted);
    (void)hipFree(c->bcnt);
    (void)hipFree(c->bfill);
    (void)hipFree(c->ctr);
    (void)hipFree(c->stats);
    (void)hipFree(c->bin_key);
    (void)hipFree(c->bin_tmp);
    (void)hipFree(c->bin_idx);
    (void)hipFree(c->binned);
    (void)hipFree(c->tbox);
    (void)hipFree(c->bin_bbox);
    (void)hipFree(c->bin_temp);
    (void)hipFree(c->partial);
    for (double *p : c->partial_retired) (void)hipFree(p);
    (void)hipFree(c->cap_dev);
    if (c->cap_pinned) (void)hipHostFree(c->cap_pinned);
    (void)hipFree(c->descs_dev);
    if (c->descs_pinned) (void)hipHostFree(c->descs_pinned);
    if (c->upload_done) (void)hipEventDestroy(c->upload_done);
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    (void)hipFree(c->enc_gp);
    (void)hipFree(c->enc_gstart);
    (void)hipFree(c->enc_gskip);
    (void)hipFree(c->enc_ctl);
    (void)hipFree(c->ingroup);
    delete c;
    return SYMBA_OK;
}

int symba_set_option(symba_ctx *c, int option, int value) {
    if (!c) return SYMBA_EINVAL;
    switch (option) {
        case SYMBA_OPT_TILE_ROWS:
            if (value != 0 && value != 1 && value != 2 && value != 4) return SYMBA_EINVAL;
            c->opt_rows = value;
            return SYMBA_OK;
        case SYMBA_OPT_FIELD_ROWS:
            if (value != 0 && value != 1 && value != 2) return SYMBA_EINVAL;
            c->opt_field_rows = value;
            return SYMBA_OK;
        case SYMBA_OPT_BIN:
            if (value < 0 || value > 2) return SYMBA_EINVAL;
            c->opt_bin = value;
            return SYMBA_OK;
        case SYMBA_OPT_TIMING:
            if (value != 0 && value != 1) return SYMBA_EINVAL;
            c->opt_timing = value;
            return SYMBA_OK;
        case SYMBA_OPT_SPLIT:
            if (value < -1 || value > kMaxSplit) return SYMBA_EINVAL;
            c->opt_split = value;
            return SYMBA_OK;
        case SYMBA_OPT_ENC_FUSE:
            if (value != 0 && value != 1) return SYMBA_EINVAL;
            c->opt_enc_fuse = value;
            return SYMBA_OK;
        case SYMBA_OPT_ENC_REGS:
            if (value != 0 && value != 1) return SYMBA_EINVAL;
            c->opt_enc_regs = value;
            return SYMBA_OK;
        case SYMBA_OPT_ACC:
            if (value != SYMBA_ACC_INTERACTION && value != SYMBA_ACC_HELIO) return SYMBA_EINVAL;
            c->opt_acc = value;
            return SYMBA_OK;
        case SYMBA_OPT_SCREEN:
            if (value != SYMBA_SCREEN_AUTO && value != SYMBA_SCREEN_FP32 && value != SYMBA_SCREEN_FP64)
                return SYMBA_EINVAL;
            c->opt_screen = value;
            return SYMBA_OK;
        default:
            return SYMBA_EINVAL;
    }
}

namespace {

// One problem through the path (single-call launches); `kick`, when not
// null, is the step's velocity arrays for the closing half kick of kick_h.
int evaluate(symba_ctx *c, const symba_state *s, int64_t n, int64_t n_m, double dt, double rcrit_factor,
             const symba_out *out, void *stream, double *const *kick, double kick_h,
             const symba::StepDesc *drifts, bool interaction_only = false) {
    const int n_tri_guess = (int)(n_m >= n - 1 ? n : n_m);
    const int rows = rows_for(c, n_tri_guess);
    const int field_rows = field_rows_for(n - n_tri_guess, c->opt_field_rows);
    const Plan p = make_plan(n, n_m, rows, field_rows, split_for(c, n_tri_guess, rows));
    int rc = grow_partial(c, p.partial_doubles, is_capturing((hipStream_t)stream));
    if (rc != SYMBA_OK) return rc;
    Desc d;
    fill_desc(d, *s, *out, n, n_m, dt, rcrit_factor, p, field_rows);
    d.task_base = 0;
    d.partial = c->partial;
    d.fpartial = d.partial + d.n_slots * 3 * d.n_tri;
    d.parent = c->parent;
    d.touched = c->touched;
    d.blk_groups = c->blk_groups;
    d.pairs = c->pairs;
    d.pair_scratch_cap = c->max_pairs;
    d.sorted = c->sorted;
    d.bcnt = c->bcnt;
    d.bfill = c->bfill;
    d.nb = symba::bucket_count(n);
    d.ctr = c->ctr;
    d.stats = c->stats;
    symba::LaunchCfg cfg{kScatterBlocks, kCloseBlocks, 0};
    d.fin_base = 0;
    if (kick) {
        d.kvx = kick[0];
        d.kvy = kick[1];
        d.kvz = kick[2];
        d.kick_h = kick_h;
    } else if (c->opt_acc == SYMBA_ACC_HELIO && !interaction_only) {
        d.ind = c->ind;
        d.n_ind = ceil_div(d.n_tri, symba::kIndBodies);
        cfg.ind_blocks = d.n_ind;
    }
    const int binned = wire_binning(c, d, use_bin(c, n, n_m), 0, 0);
    const symba::TileGroup g{rows, field_rows, binned, screen32(c), 0, 1, 0, d.n_tasks};
    if (drifts && symba::launch_drifts(*drifts, nullptr, 0, drifts->nblk, (hipStream_t)stream) != hipSuccess)
        return SYMBA_EDEVICE;
    hipError_t e = symba::launch_step(&d, nullptr, 1, &g, 1, binned, symba::final_blocks(n, kScatterBlocks), cfg,
                                      (hipStream_t)stream, timing_slot(c));
    return e == hipSuccess ? SYMBA_OK : SYMBA_EDEVICE;
}

}  // namespace

int symba_kick_encounter(symba_ctx *c, const symba_state *s, int64_t n, int64_t n_m, double dt,
                         double rcrit_factor, const symba_out *out, void *stream) {
    if (!c || bad_state(s) || bad_out(out)) return SYMBA_EINVAL;
    if (n < 1 || n_m < 0 || n_m > n || bad_scalar(dt, rcrit_factor)) return SYMBA_EINVAL;
    if (n > c->max_n) return SYMBA_ETOOBIG;
    if (hipSetDevice(c->device) != hipSuccess) return SYMBA_EDEVICE;
    return evaluate(c, s, n, n_m, dt, rcrit_factor, out, stream, nullptr, 0.0, nullptr);
}

}  // extern "C"

// Scratch of symba_kick_encounter_noalloc: one fixed region per device, in
// the library's own device memory (loaded with the code object, held until
// the process ends), carved like a context's scratch for problems of up to
// SYMBA_NOALLOC_MAX_N bodies and SYMBA_NOALLOC_MAX_PAIRS stored pairs.  The
// first part must be zero between calls (the kernels leave it so); it is
// zeroed once per device, by a kernel on the first call's stream.
namespace {

constexpr int64_t kNoallocMaxN = SYMBA_NOALLOC_MAX_N;
constexpr int64_t kNoallocMaxPairs = SYMBA_NOALLOC_MAX_PAIRS;
constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
// partial-sum slots for n <= kNoallocMaxN with the default options: at
// n_tri >= 4000 two bodies per lane, at most n / 128 blocks of 128 bodies
// plus 2 (R - 1) = 2 per split diagonal (at most kMaxSplit); below 4000 one
// body per lane, at most 63 blocks of 64 over fewer than 4000 bodies (less
// in all).  A plan that needed more would be refused (SYMBA_ETOOBIG).
constexpr size_t kNoallocSlots = kNoallocMaxN / 128 + 2 * kMaxSplit;
constexpr size_t kNzParent = 0;
constexpr size_t kNzTouched = kNzParent + align256(sizeof(int32_t) * kNoallocMaxN);
constexpr size_t kNzBcnt = kNzTouched + align256(sizeof(int32_t) * kNoallocMaxN);
constexpr size_t kNzBfill = kNzBcnt + align256(sizeof(int32_t) * kNoallocMaxN);
constexpr size_t kNzCtr = kNzBfill + align256(sizeof(int32_t) * kNoallocMaxN);
constexpr size_t kNzStats = kNzCtr + align256(sizeof(unsigned long long) * symba::kCtrSlots);
constexpr size_t kNzEnd = kNzStats + align256(sizeof(unsigned long long) * symba::kStatSlots);  // zero part
constexpr size_t kNoBlkGroups = kNzEnd;
constexpr size_t kNoPairs = kNoBlkGroups + align256(sizeof(int32_t) * (kNoallocMaxN / symba::kFinBodies + 1));
constexpr size_t kNoSorted = kNoPairs + align256(sizeof(int2) * kNoallocMaxPairs);
constexpr size_t kNoPartial = kNoSorted + align256(sizeof(int4) * kNoallocMaxPairs);
constexpr size_t kNoPartialBytes = sizeof(double) * kNoallocSlots * 3 * kNoallocMaxN;
constexpr size_t kNoallocBytes = kNoPartial + kNoPartialBytes;
static_assert(kNoallocBytes == SYMBA_NOALLOC_SCRATCH_BYTES, "symba.h states the scratch size");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

constexpr int kNoallocDevices = 64;
std::mutex g_noalloc_mutex;
unsigned char *g_noalloc_ptr[kNoallocDevices] = {};  // device address of `scratch`, per device
bool g_noalloc_zeroed[kNoallocDevices] = {};

// The device address of this device's `scratch` (the host-side name is only a
// stand-in for it), found once per device with that device current.
int noalloc_scratch(int device, unsigned char **ptr, bool *first) {
    if (device < 0 || device >= kNoallocDevices) return SYMBA_EDEVICE;
    std::lock_guard<std::mutex> lock(g_noalloc_mutex);
    if (!g_noalloc_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SYMBA_EDEVICE;
        g_noalloc_ptr[device] = (unsigned char *)p;
    }
    *ptr = g_noalloc_ptr[device];
    *first = !g_noalloc_zeroed[device];
    g_noalloc_zeroed[device] = true;
    return SYMBA_OK;
}

}  // namespace

extern "C" {

int symba_kick_encounter_noalloc(const symba_state *s, int64_t n, int64_t n_m, double dt, double rcrit_factor,
                                 const symba_out *out, void *stream) {
    if (bad_state(s) || bad_out(out)) return SYMBA_EINVAL;
    if (n < 1 || n_m < 0 || n_m > n || bad_scalar(dt, rcrit_factor)) return SYMBA_EINVAL;
    if (n > kNoallocMaxN) return SYMBA_ETOOBIG;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return SYMBA_EDEVICE;
    unsigned char *base = nullptr;
    bool first = false;
    int rc = noalloc_scratch(device, &base, &first);
    if (rc != SYMBA_OK) return rc;
    if (first && symba::launch_zero(base, kNzEnd, (hipStream_t)stream) != hipSuccess) {
        std::lock_guard<std::mutex> lock(g_noalloc_mutex);
        g_noalloc_zeroed[device] = false;
        return SYMBA_EDEVICE;
    }
    symba_ctx c;  // a view of the fixed region: owns nothing, frees nothing
    c.device = device;
    c.max_n = kNoallocMaxN;
    c.max_pairs = kNoallocMaxPairs;
    c.max_problems = 1;
    c.fixed_scratch = true;
    c.parent = (int32_t *)(base + kNzParent);
    c.touched = (int32_t *)(base + kNzTouched);
    c.bcnt = (int32_t *)(base + kNzBcnt);
    c.bfill = (int32_t *)(base + kNzBfill);
    c.ctr = (unsigned long long *)(base + kNzCtr);
    c.stats = (unsigned long long *)(base + kNzStats);
    c.blk_groups = (int32_t *)(base + kNoBlkGroups);
    c.pairs = (int2 *)(base + kNoPairs);
    c.sorted = (int4 *)(base + kNoSorted);
    c.partial = (double *)(base + kNoPartial);
    c.partial_bytes = kNoPartialBytes;
    return evaluate(&c, s, n, n_m, dt, rcrit_factor, out, stream, nullptr, 0.0, nullptr);
}

int symba_step(symba_ctx *c, const symba_mstate *s, int64_t n, int64_t n_m, double h, double rcrit_factor,
               const symba_out *out, void *stream) {
    if (!c || !s || !s->x || !s->y || !s->z || !s->vx || !s->vy || !s->vz || !s->m || !s->rh || bad_out(out))
        return SYMBA_EINVAL;
    if (n < 1 || n_m < 0 || n_m > n || !std::isfinite(h) || bad_scalar(std::fabs(h), rcrit_factor))
        return SYMBA_EINVAL;
    if (n > c->max_n) return SYMBA_ETOOBIG;
    if (hipSetDevice(c->device) != hipSuccess) return SYMBA_EDEVICE;
    symba::StepDesc sd{};
    sd.x = s->x; sd.y = s->y; sd.z = s->z; sd.vx = s->vx; sd.vy = s->vy; sd.vz = s->vz; sd.m = s->m;
    sd.ax = out->ax; sd.ay = out->ay; sd.az = out->az;
    sd.n = n;
    sd.n_tri = n_m >= n - 1 ? n : n_m;
    sd.kick_h = 0.5 * h;
    sd.sun_h = 0.5 * h;
    sd.kepler_h = h;
    sd.mom0 = c->mom;
    sd.mom1 = c->mom + 3 * c->mom_blocks;
    sd.blk_base = 0;
    sd.nblk = symba::step_blocks(n);
    const symba_state cs{s->x, s->y, s->z, s->vx, s->vy, s->vz, s->m, s->rh};
    double *const kick[3] = {s->vx, s->vy, s->vz};
    return evaluate(c, &cs, n, n_m, std::fabs(h), rcrit_factor, out, stream, kick, 0.5 * h, &sd);
}

namespace {

// The encounter step's view of a state, its outputs and the context's table.
symba::EncDesc enc_desc(symba_ctx *c, const symba_mstate *s, int64_t n, int64_t n_m, double h, double f,
                        const symba_out *out) {
    symba::EncDesc e{};
    e.x = s->x; e.y = s->y; e.z = s->z; e.vx = s->vx; e.vy = s->vy; e.vz = s->vz; e.m = s->m; e.rh = s->rh;
    e.ax = out->ax; e.ay = out->ay; e.az = out->az;
    e.n = n;
    e.n_tri = n_m >= n - 1 ? n : n_m;
    e.f = f;
    e.h = h;
    e.kick_h = 0.5 * h;
    e.pair_i = out->pair_i; e.pair_j = out->pair_j; e.n_pairs = out->n_pairs; e.status = out->status;
    e.group_id = out->group_id;
    e.pair_cap = out->pair_cap;
    e.gp = c->enc_gp; e.gstart = c->enc_gstart; e.gskip = c->enc_gskip; e.ctl = c->enc_ctl;
    e.ingroup = c->ingroup;
    e.regs = c->opt_enc_regs;
    return e;
}

bool bad_mstate(const symba_mstate *s) {
    return !s || !s->x || !s->y || !s->z || !s->vx || !s->vy || !s->vz || !s->m || !s->rh;
}

// Problems of one drift block take the fused encounter launches.
bool enc_fused(const symba_ctx *c, int64_t n) { return c->opt_enc_fuse && symba::step_blocks(n) == 1; }

// Level-0 reweighting of the evaluation in `out` (pairs, groups and
// Newtonian accelerations at s), then the closing kick when e.kick_h != 0.
int enc_finish(const symba_ctx *c, symba::EncDesc e, hipStream_t stream) {
    e.mark = 0;
    if (enc_fused(c, e.n)) return symba::launch_enc_post_block(e, stream) == hipSuccess ? SYMBA_OK : SYMBA_EDEVICE;
    if (symba::launch_enc_table(e, stream) != hipSuccess || symba::launch_enc_level0(e, stream) != hipSuccess ||
        symba::launch_enc_kick(e, stream) != hipSuccess)
        return SYMBA_EDEVICE;
    return SYMBA_OK;
}

}  // namespace

int symba_enc_prepare(symba_ctx *c, const symba_mstate *s, int64_t n, int64_t n_m, double h, double rcrit_factor,
                      const symba_out *out, void *stream) {
    if (!c || bad_mstate(s) || bad_out(out)) return SYMBA_EINVAL;
    if (n < 1 || n_m < 0 || n_m > n || !std::isfinite(h) || bad_scalar(std::fabs(h), rcrit_factor))
        return SYMBA_EINVAL;
    if (n > c->max_n) return SYMBA_ETOOBIG;
    if (hipSetDevice(c->device) != hipSuccess) return SYMBA_EDEVICE;
    const symba_state cs{s->x, s->y, s->z, s->vx, s->vy, s->vz, s->m, s->rh};
    int rc = evaluate(c, &cs, n, n_m, std::fabs(h), rcrit_factor, out, stream, nullptr, 0.0, nullptr, true);
    if (rc != SYMBA_OK) return rc;
    symba::EncDesc e = enc_desc(c, s, n, n_m, h, rcrit_factor, out);
    e.kick_h = 0.0;
    return enc_finish(c, e, (hipStream_t)stream);
}

int symba_step_enc(symba_ctx *c, const symba_mstate *s, int64_t n, int64_t n_m, double h, double rcrit_factor,
                   const symba_out *out, void *stream) {
    if (!c || bad_mstate(s) || bad_out(out)) return SYMBA_EINVAL;
    if (n < 1 || n_m < 0 || n_m > n || !std::isfinite(h) || bad_scalar(std::fabs(h), rcrit_factor))
        return SYMBA_EINVAL;
    if (n > c->max_n) return SYMBA_ETOOBIG;
    if (hipSetDevice(c->device) != hipSuccess) return SYMBA_EDEVICE;
    symba::StepDesc sd{};
    sd.x = s->x; sd.y = s->y; sd.z = s->z; sd.vx = s->vx; sd.vy = s->vy; sd.vz = s->vz; sd.m = s->m;
    sd.ax = out->ax; sd.ay = out->ay; sd.az = out->az;
    sd.n = n;
    sd.n_tri = n_m >= n - 1 ? n : n_m;
    sd.kick_h = 0.5 * h;
    sd.sun_h = 0.5 * h;
    sd.kepler_h = h;
    sd.mom0 = c->mom;
    sd.mom1 = c->mom + 3 * c->mom_blocks;
    sd.blk_base = 0;
    sd.nblk = symba::step_blocks(n);
    sd.skip = c->ingroup;
    symba::EncDesc e = enc_desc(c, s, n, n_m, h, rcrit_factor, out);
    e.mark = 1;
    const hipStream_t st = (hipStream_t)stream;
    const hipError_t de = enc_fused(c, n) ? symba::launch_enc_drifts_block(sd, e, st)
                                          : symba::launch_drifts_enc(sd, e, st);
    if (de != hipSuccess) return SYMBA_EDEVICE;
    const symba_state cs{s->x, s->y, s->z, s->vx, s->vy, s->vz, s->m, s->rh};
    int rc = evaluate(c, &cs, n, n_m, std::fabs(h), rcrit_factor, out, stream, nullptr, 0.0, nullptr, true);
    if (rc != SYMBA_OK) return rc;
    return enc_finish(c, e, st);
}

namespace {

// The batch evaluation; with `steps` (the same problems as steps, in the same
// order) the drifts run first and each problem's final kernel applies the
// closing half kick.
int batch_impl(symba_ctx *c, const symba_problem *probs, int32_t n_problems, void *stream,
               const symba_step_problem *steps) {
    int64_t total_n = 0;
    for (int32_t k = 0; k < n_problems; ++k) {
        const symba_problem &q = probs[k];
        if (bad_state(&q.state) || bad_out(&q.out)) return SYMBA_EINVAL;
        if (q.n < 1 || q.n_m < 0 || q.n_m > q.n || bad_scalar(q.dt, q.rcrit_factor)) return SYMBA_EINVAL;
        total_n += q.n;
    }
    if (total_n > c->max_n) return SYMBA_ETOOBIG;
    if (hipSetDevice(c->device) != hipSuccess) return SYMBA_EDEVICE;
    // Each problem gets the tile size a single call would give it, so its
    // results do not depend on the rest of the batch; problems are ordered by
    // tile size and each size is one tile-kernel launch.
    std::vector<int> rows((size_t)n_problems), frows((size_t)n_problems), bins((size_t)n_problems),
        order((size_t)n_problems);
    for (int32_t k = 0; k < n_problems; ++k) {
        const symba_problem &q = probs[k];
        const int64_t n_tri = q.n_m >= q.n - 1 ? q.n : q.n_m;
        rows[k] = rows_for(c, n_tri);
        frows[k] = field_rows_for(q.n - n_tri, c->opt_field_rows);
        bins[k] = use_bin(c, q.n, q.n_m) ? 1 : 0;
        order[k] = k;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (rows[a] != rows[b]) return rows[a] < rows[b];
        if (frows[a] != frows[b]) return frows[a] < frows[b];
        return bins[a] < bins[b];
    });
    std::vector<Desc> ds((size_t)n_problems);
    std::vector<Plan> plans((size_t)n_problems);
    std::vector<symba::TileGroup> groups;
    size_t partial_total = 0;
    for (int32_t s = 0; s < n_problems; ++s) {
        const symba_problem &q = probs[order[s]];
        const int64_t n_tri = q.n_m >= q.n - 1 ? q.n : q.n_m;
        plans[s] = make_plan(q.n, q.n_m, rows[order[s]], frows[order[s]], split_for(c, n_tri, rows[order[s]]));
        partial_total += plans[s].partial_doubles;
    }
    hipStream_t st = (hipStream_t)stream;
    const bool capturing = is_capturing(st);
    int rc = grow_partial(c, partial_total, capturing);
    if (rc != SYMBA_OK) return rc;
    int64_t task_total = 0, fin_total = 0, body_off = 0, blk_off = 0, pair_off = 0, box_off = 0, ind_off = 0;
    int n_binned = 0;
    size_t partial_off = 0;
    symba::LaunchCfg cfg{kScatterBlocksBatch, kCloseBlocksBatch, 0};
    for (int32_t s = 0; s < n_problems; ++s) {
        const int k = order[s];
        const symba_problem &q = probs[k];
        if (groups.empty() || groups.back().rows != rows[k] || groups.back().field_rows != frows[k] ||
            groups.back().binned != bins[k])
            groups.push_back(symba::TileGroup{rows[k], frows[k], bins[k], screen32(c), s, s, task_total, 0});
        Desc &d = ds[s];
        fill_desc(d, q.state, q.out, q.n, q.n_m, q.dt, q.rcrit_factor, plans[s], frows[k]);
        if (steps) {
            d.kvx = steps[k].state.vx;
            d.kvy = steps[k].state.vy;
            d.kvz = steps[k].state.vz;
            d.kick_h = 0.5 * steps[k].h;
        } else if (c->opt_acc == SYMBA_ACC_HELIO) {
            d.ind = c->ind + 3 * ind_off;
            d.n_ind = ceil_div(d.n_tri, symba::kIndBodies);
            d.ind_base = ind_off;
            ind_off += d.n_ind;
        }
        d.task_base = task_total;
        d.partial = c->partial + partial_off;
        d.fpartial = d.partial + d.n_slots * 3 * d.n_tri;
        d.parent = c->parent + body_off;
        d.touched = c->touched + body_off;
        d.blk_groups = c->blk_groups + blk_off;
        const int64_t share = std::min<int64_t>(std::max<int64_t>(q.out.pair_cap, 0), c->max_pairs - pair_off);
        d.pairs = c->pairs + pair_off;
        d.sorted = c->sorted + pair_off;
        d.bcnt = c->bcnt + body_off;
        d.bfill = c->bfill + body_off;
        d.nb = symba::bucket_count(q.n);
        d.pair_scratch_cap = share;
        d.ctr = c->ctr + symba::kCtrSlots * (int64_t)s;
        d.stats = c->stats;
        d.fin_base = fin_total;
        n_binned += wire_binning(c, d, bins[k] != 0, body_off, box_off);
        box_off += d.n_boxes;
        task_total += d.n_tasks;
        fin_total += symba::final_blocks(q.n, kScatterBlocksBatch);
        body_off += q.n;
        blk_off += plans[s].n_blk;
        pair_off += share;
        partial_off += plans[s].partial_doubles;
        groups.back().p1 = s + 1;
        groups.back().n_tasks += d.n_tasks;
    }
    cfg.ind_blocks = ind_off;
    if (steps) {  // the drift descriptors, in the caller's order, each problem a range of blocks
        if (!capturing && c->steps_pending && hipEventSynchronize(c->steps_done) != hipSuccess)
            return SYMBA_EDEVICE;
        std::vector<symba::StepDesc> sds((size_t)n_problems);
        int64_t blk = 0;
        for (int32_t k = 0; k < n_problems; ++k) {
            const symba_step_problem &q = steps[k];
            symba::StepDesc &sd = sds[k];
            sd = symba::StepDesc{};
            sd.x = q.state.x; sd.y = q.state.y; sd.z = q.state.z;
            sd.vx = q.state.vx; sd.vy = q.state.vy; sd.vz = q.state.vz; sd.m = q.state.m;
            sd.ax = q.out.ax; sd.ay = q.out.ay; sd.az = q.out.az;
            sd.n = q.n;
            sd.n_tri = q.n_m >= q.n - 1 ? q.n : q.n_m;
            sd.kick_h = 0.5 * q.h;
            sd.sun_h = 0.5 * q.h;
            sd.kepler_h = q.h;
            sd.mom0 = c->mom;
            sd.mom1 = c->mom + 3 * c->mom_blocks;
            sd.blk_base = blk;
            sd.nblk = symba::step_blocks(q.n);
            blk += sd.nblk;
        }
        const size_t sbytes = sizeof(symba::StepDesc) * n_problems;
        symba::StepDesc *steps_dev = c->steps_dev;
        if (capturing) {  // descriptors of its own, which no later call rewrites
            steps_dev = (symba::StepDesc *)capture_upload(c, sds.data(), sbytes, st);
            if (!steps_dev) return SYMBA_ENOMEM;
        } else {
            std::memcpy(c->steps_pinned, sds.data(), sbytes);
            if (hipMemcpyAsync(c->steps_dev, c->steps_pinned, sbytes, hipMemcpyHostToDevice, st) != hipSuccess ||
                hipEventRecord(c->steps_done, st) != hipSuccess)
                return SYMBA_EDEVICE;
            c->steps_pending = true;
        }
        if (symba::launch_drifts(sds[0], steps_dev, n_problems, blk, st) != hipSuccess) return SYMBA_EDEVICE;
    }
    const Desc *descs_dev = c->descs_dev;
    if (capturing) {  // descriptors of its own, which no later call rewrites
        descs_dev = (const Desc *)capture_upload(c, ds.data(), sizeof(Desc) * ds.size(), st);
        if (!descs_dev) return SYMBA_ENOMEM;
    } else {
        const bool same = c->descs_last.size() == ds.size() &&
                          std::memcmp(c->descs_last.data(), ds.data(), sizeof(Desc) * ds.size()) == 0;
        if (!same) {
            if (c->upload_pending && hipEventSynchronize(c->upload_done) != hipSuccess) return SYMBA_EDEVICE;
            std::memcpy(c->descs_pinned, ds.data(), sizeof(Desc) * ds.size());
            if (hipMemcpyAsync(c->descs_dev, c->descs_pinned, sizeof(Desc) * ds.size(), hipMemcpyHostToDevice,
                               st) != hipSuccess)
                return SYMBA_EDEVICE;
            if (hipEventRecord(c->upload_done, st) != hipSuccess) return SYMBA_EDEVICE;
            c->upload_pending = true;
            c->descs_last = ds;
        }
    }
    hipError_t e = symba::launch_step(ds.data(), descs_dev, n_problems, groups.data(), (int)groups.size(),
                                      n_binned, fin_total, cfg, st, capturing ? nullptr : timing_slot(c));
    return e == hipSuccess ? SYMBA_OK : SYMBA_EDEVICE;
}

}  // namespace

int symba_kick_encounter_batch(symba_ctx *c, const symba_problem *probs, int32_t n_problems,
                               void *stream) {
    if (!c || !probs || n_problems < 1 || n_problems > c->max_problems) return SYMBA_EINVAL;
    return batch_impl(c, probs, n_problems, stream, nullptr);
}

int symba_step_batch(symba_ctx *c, const symba_step_problem *steps, int32_t n_problems, void *stream) {
    if (!c || !steps || n_problems < 1 || n_problems > c->max_problems) return SYMBA_EINVAL;
    std::vector<symba_problem> probs((size_t)n_problems);
    for (int32_t k = 0; k < n_problems; ++k) {
        const symba_step_problem &q = steps[k];
        const symba_mstate &m = q.state;
        if (!m.x || !m.y || !m.z || !m.vx || !m.vy || !m.vz || !m.m || !m.rh || !std::isfinite(q.h))
            return SYMBA_EINVAL;
        probs[k].state = symba_state{m.x, m.y, m.z, m.vx, m.vy, m.vz, m.m, m.rh};
        probs[k].n = q.n;
        probs[k].n_m = q.n_m;
        probs[k].dt = std::fabs(q.h);
        probs[k].rcrit_factor = q.rcrit_factor;
        probs[k].out = q.out;
    }
    return batch_impl(c, probs.data(), n_problems, stream, steps);
}

int symba_read_timing(symba_ctx *c, double *tiles_ms, double *finalize_ms, int64_t *calls) {
    if (!c) return SYMBA_EINVAL;
    double t = 0.0, fz = 0.0;
    for (size_t k = 0; k < c->timed_calls; ++k) {
        hipEvent_t *ev = c->events.data() + 3 * k;
        float a = 0.f, b = 0.f;
        if (hipEventSynchronize(ev[2]) != hipSuccess || hipEventElapsedTime(&a, ev[0], ev[1]) != hipSuccess ||
            hipEventElapsedTime(&b, ev[1], ev[2]) != hipSuccess)
            return SYMBA_EDEVICE;
        t += a;
        fz += b;
    }
    if (tiles_ms) *tiles_ms = t;
    if (finalize_ms) *finalize_ms = fz;
    if (calls) *calls = (int64_t)c->timed_calls;
    c->timed_calls = 0;
    return SYMBA_OK;
}

int64_t symba_plan_tasks(int64_t n, int64_t n_m, int32_t rows, int32_t field_rows, int64_t *tasks,
                         int64_t cap) {
    if (n < 1 || n_m < 0 || n_m > n || (rows != 1 && rows != 2 && rows != 4) ||
        (field_rows != 1 && field_rows != 2) || cap < 0 || (cap > 0 && !tasks))
        return -1;
    const Plan p = make_plan(n, n_m, rows, field_rows, -1);
    const int64_t total = p.n_tri_tasks + p.n_field_tasks;
    for (int64_t f = 0; f < std::min(total, cap); ++f) {
        const int64_t t = symba::task_in_order(p.n_tri_tasks, total, f);
        if (t < p.n_whole) {
            int64_t I, J;
            symba::whole_decode(p.B, p.n_split, t, I, J);
            tasks[3 * f] = 0;
            tasks[3 * f + 1] = I;
            tasks[3 * f + 2] = J;
        } else if (t < p.n_tri_tasks) {
            const symba::SplitTask T = symba::split_decode(p.B, rows, t - p.n_whole);
            tasks[3 * f] = 2;
            tasks[3 * f + 1] = T.I * rows + T.r;
            tasks[3 * f + 2] = T.J * rows + T.q;
        } else {
            int64_t fb, sg;
            symba::field_decode(p.n_fblocks, p.n_fslots, t - p.n_tri_tasks, fb, sg);
            tasks[3 * f] = 1;
            tasks[3 * f + 1] = fb;
            tasks[3 * f + 2] = sg;
        }
    }
    return total;
}

int symba_read_stats(symba_ctx *c, int64_t *candidates, int64_t *flagged, int64_t *problems) {
    if (!c) return SYMBA_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return SYMBA_EDEVICE;
    unsigned long long h[symba::kStatSlots] = {};
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(h, c->stats, sizeof h, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemset(c->stats, 0, sizeof h) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return SYMBA_EDEVICE;
    int64_t cand = 0;
    for (int k = 0; k < symba::kStatCandLanes; ++k) cand += (int64_t)h[symba::kStatCandidates + k];
    if (candidates) *candidates = cand;
    if (flagged) *flagged = (int64_t)h[symba::kStatFlagged];
    if (problems) *problems = (int64_t)h[symba::kStatCalls];
    return SYMBA_OK;
}

int symba_autotune(symba_ctx *c, const symba_state *s, int64_t n, int64_t n_m, double dt, double rcrit_factor,
                   const symba_out *out, void *stream, int32_t *chosen_rows) {
    if (!c || bad_state(s) || bad_out(out)) return SYMBA_EINVAL;
    if (n < 1 || n_m < 0 || n_m > n || bad_scalar(dt, rcrit_factor)) return SYMBA_EINVAL;
    if (n > c->max_n) return SYMBA_ETOOBIG;
    const int64_t n_tri = n_m >= n - 1 ? n : n_m;
    if (std::min(n_m, n - 1) < 1) {  // no pairs: nothing to tune
        if (chosen_rows) *chosen_rows = rows_for(c, n_tri);
        return symba_kick_encounter(c, s, n, n_m, dt, rcrit_factor, out, stream);
    }
    if (hipSetDevice(c->device) != hipSuccess) return SYMBA_EDEVICE;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return SYMBA_EDEVICE;
    }
    const int saved_rows = c->opt_rows, saved_timing = c->opt_timing, saved_split = c->opt_split;
    c->opt_timing = 0;
    // tile sizes, and with 2 or 4 rows the fold's tail split: 0 to 3 split
    // diagonals (distinct plans only: the fold clamps what it cannot split)
    constexpr int kRows[3] = {1, 2, 4};
    constexpr int kReps = 3;
    int best = 0, best_split = 0, rc = SYMBA_OK;
    float best_ms = 0.f;
    for (int r : kRows) {
        const int64_t B = (n_tri + (int64_t)r * symba::kWave - 1) / ((int64_t)r * symba::kWave);
        for (int D = 0; D <= 3 && rc == SYMBA_OK; ++D) {
            if (D > 0 && symba::split_diagonals(B, r, D) < D) break;
            c->opt_rows = r;
            c->opt_split = D;
            rc = symba_kick_encounter(c, s, n, n_m, dt, rcrit_factor, out, stream);  // warm-up, buffer growth
            if (rc != SYMBA_OK) break;
            float ms = 0.f;
            if (hipEventRecord(e0, st) != hipSuccess) { rc = SYMBA_EDEVICE; break; }
            for (int k = 0; k < kReps && rc == SYMBA_OK; ++k)
                rc = symba_kick_encounter(c, s, n, n_m, dt, rcrit_factor, out, stream);
            if (rc != SYMBA_OK) break;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = SYMBA_EDEVICE;
                break;
            }
            if (best == 0 || ms < best_ms) {
                best = r;
                best_split = D;
                best_ms = ms;
            }
        }
        if (rc != SYMBA_OK) break;
    }
    c->opt_rows = saved_rows;
    c->opt_timing = saved_timing;
    c->opt_split = saved_split;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SYMBA_OK) return rc;
    c->tuned_rows[size_class(n_tri)] = best;
    c->tuned_split[size_class(n_tri)] = best_split + 1;
    if (chosen_rows) *chosen_rows = best;
    // leave the problem's outputs as a call with the tuned size writes them
    return symba_kick_encounter(c, s, n, n_m, dt, rcrit_factor, out, stream);
}

int symba_plan_for(const symba_ctx *c, int64_t n, int64_t n_m, int32_t *rows, int32_t *split) {
    if (!c || n < 1 || n_m < 0 || n_m > n) return SYMBA_EINVAL;
    const int64_t n_tri = n_m >= n - 1 ? n : n_m;
    const int r = rows_for(c, n_tri);
    const Plan p = make_plan(n, n_m, r, field_rows_for(n - n_tri, c->opt_field_rows), split_for(c, n_tri, r));
    if (rows) *rows = r;
    if (split) *split = (int32_t)p.n_split;
    return SYMBA_OK;
}

int64_t symba_scratch_bytes(const symba_ctx *c, int64_t n, int64_t n_m, int64_t pair_cap) {
    if (!c || n < 1 || n_m < 0 || n_m > n || pair_cap < 0) return -1;
    const int64_t n_tri = n_m >= n - 1 ? n : n_m;
    const int rows = rows_for(c, n_tri);
    const Plan p = make_plan(n, n_m, rows, field_rows_for(n - n_tri, c->opt_field_rows), split_for(c, n_tri, rows));
    const int64_t per_body = 5 * (int64_t)sizeof(int32_t) +                                 // parent, touched, buckets
                             (use_bin(c, n, n_m) ? 3 * (int64_t)sizeof(int32_t) + 8 * (int64_t)sizeof(double) +
                                                       symba::kBoxDoubles * (int64_t)sizeof(double) / symba::kWave
                                                 : 0);  // binning
    const int64_t per_pair = (int64_t)sizeof(int2) + (int64_t)sizeof(int4);            // pair lists
    return (int64_t)(p.partial_doubles * sizeof(double)) + per_body * n + per_pair * pair_cap +
           (int64_t)sizeof(int32_t) * p.n_blk +  // groups per final-kernel body block
           (int64_t)sizeof(Desc);
}

}  // extern "C"
