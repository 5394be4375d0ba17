// C ABI of the library: context lifetime, workspace layout, the one-time
// set-up of Algorithm 1 (first three lines) and the per-block loop of
// Algorithm 2 with double-buffered host-to-device copies on side streams.
#include "gwas.h"
#include "internal.h"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

using namespace gwas;

namespace {

constexpr uint64_t CTX_MAGIC = 0x67776173c7c70001ull;
constexpr uint64_t CTX_DEAD = 0xdeadc7c7deadc7c7ull;
constexpr int64_t DEFAULT_DEV_BLOCK = 16384;
constexpr int MAX_T = 256;
constexpr double RANK_TOL_F64 = 1e-10;
constexpr double RANK_TOL_F32 = 1e-6;
constexpr double RANK_TOL_BF16 = 1e-2;
constexpr double RANK_TOL_I8S = 1e-10;
constexpr int DEFAULT_SLICES = 6;
constexpr int REFINE_STEPS = 2;

struct Layout {
    int64_t n, n_pad, ld, dev_block, npb_max, Q;
    // banded M: half-bandwidth (0 = dense), block order W and block rows nb;
    // the factor is kept as U_ii = L_ii^-T and Gt_i = -E_i^T U_ii per block row
    int64_t band, W, nb, band_ld;
    size_t off_bandcopy;
    size_t off_Ub, off_Gt, off_Ab, off_Eb, off_Z[2];
    int p, t, q1, Qc, precision, x_dtype, slices;
    size_t off_L, off_U, off_Ulow, off_rscale, off_rsum, off_XY, off_C, off_W, off_S, off_consts, off_flags,
        off_sched, off_sched_tail, off_region;
    size_t off_xbuf[2], off_part, off_red, off_xw, off_xwpart, off_xsl, off_b[2], off_v[2], off_i[2];
    size_t off_tmp;
    size_t sched_len;
    // gwas_stream_block_noalloc: sub-block width whose per-SNP scratch fits
    // the static device buffer (0: not even one column tile fits), and the
    // room of its tile schedule in the workspace
    int64_t na_cols;
    size_t na_sched_len, off_sched_na;
    size_t total;
};

// The static device buffer of gwas_stream_block_noalloc.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(256) << 20;
constexpr size_t NOALLOC_ALIGN = 256;

// The product's dosage operand: the dosages as handed over, or float64
// dosages cut once per sub-block into bfloat16 for the bfloat16 products
// (three slices for the bfloat16-slice mode, one rounding for the bfloat16
// mode).
int prod_xt_of(int precision, int x_dtype) {
    if (x_dtype == GWAS_X_I8) return X_I8;
    if (precision == GWAS_BF16X3_REFINE) return X_BF16S;
    return precision == GWAS_BF16_REFINE ? X_BF16 : X_F64;
}
bool x_cut(int xt) { return xt == X_BF16S || xt == X_BF16; }
// elements per column of the cut dosages (their leading dimension)
int64_t x_cut_ld(int xt, int64_t n_pad) { return xt == X_BF16S ? 3 * n_pad : n_pad; }

// Offsets, in a buffer of per-SNP scratch for `cols` columns, of the
// product's partial sums, their chunk totals, (reduced modes) the cross
// products x^T W with their split-K partials and (bfloat16 products with
// float64 dosages) the cut dosages; [5] is the end.
void noalloc_offsets(const Layout& L, int64_t cols, size_t off[6]) {
    const bool red = L.precision != GWAS_FP64;
    const int xt = prod_xt_of(L.precision, L.x_dtype);
    const size_t sz[5] = {
        (size_t)L.npb_max * L.Q * cols * 8, (size_t)chunks_of(L.npb_max) * L.Q * cols * 8,
        red ? (size_t)L.Qc * cols * 8 : 0, red ? (size_t)xw_splits(L.n) * L.Qc * cols * 8 : 0,
        x_cut(xt) ? (size_t)x_cut_ld(xt, L.n_pad) * cols * x_elem_bytes(xt) : 0};
    size_t o = 0;
    for (int i = 0; i < 5; ++i) {
        off[i] = o;
        o = (o + sz[i] + NOALLOC_ALIGN - 1) / NOALLOC_ALIGN * NOALLOC_ALIGN;
    }
    off[5] = o;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

constexpr int64_t BAND_MAX_N_F64 = 2000000, BAND_MAX_N_I8 = 16000000;
constexpr int64_t INT8_SLICED_MAX_N = 260096;     // a multiple of 256

bool sizes_valid(int64_t n, int32_t p, int32_t t, int64_t dev_block, int32_t precision,
                 int32_t x_dtype, int64_t band = 0) {
    if (band < 0 || (band > 0 && precision != GWAS_FP64)) return false;
    if (p < 2 || p > 20 || n < p || t < 1 || t > MAX_T) return false;
    if (n > (int64_t)1 << 24) return false;
    if (dev_block < 0 || dev_block > ((int64_t)1 << 22)) return false;
    if (precision < GWAS_FP64 || precision > GWAS_BF16X3_REFINE) return false;
    if (x_dtype != GWAS_X_F64 && x_dtype != GWAS_X_I8) return false;
    if (precision == GWAS_INT8_SLICED && x_dtype != GWAS_X_I8) return false;
    // exact int32 sums of the paired digits against the dosages
    // (|127 A_hi (x - 1) + A_lo x| <= 8,256 per element) need
    // 8,256 n_pad < 2^31
    if (precision == GWAS_INT8_SLICED && n > INT8_SLICED_MAX_N) return false;
    // the banded product addresses 128 dosage columns of a tile with 32-bit
    // offsets: 128 n_pad bytes of int8, 1,024 n_pad of float64, below 2^31
    if (band > 0 && n > (x_dtype == GWAS_X_F64 ? BAND_MAX_N_F64 : BAND_MAX_N_I8)) return false;
    return true;
}

int atype_of(int precision) {
    return precision == GWAS_FP64 ? A_F64 : precision == GWAS_FP32_REFINE ? A_F32
         : (precision == GWAS_BF16_REFINE || precision == GWAS_BF16X3_REFINE) ? A_BF16 : A_I8S;
}

// Block order of a banded M of half-bandwidth w: a multiple of 256 rows at
// least w, so that M is block tridiagonal.
int64_t band_block_order(int64_t w) { return (w + 255) / 256 * 256; }

Layout make_layout(int64_t n, int p, int t, int64_t dev_block, int precision, int x_dtype,
                   int slices, int64_t band = 0, int64_t band_ld = 0) {
    Layout L{};
    L.band = band;
    L.band_ld = band > 0 ? std::max(band_ld, band + 1) : 0;
    L.W = band > 0 ? band_block_order(band) : 0;
    // int8 digits of L^-1, or its three bfloat16 slices
    L.slices = precision == GWAS_INT8_SLICED ? slices : precision == GWAS_BF16X3_REFINE ? 3 : 0;
    L.n = n;
    L.p = p;
    L.t = t;
    L.q1 = p - 1;
    L.Qc = p - 1 + t;
    L.precision = precision;
    L.x_dtype = x_dtype;
    L.n_pad = (n + NPAD_ALIGN - 1) / NPAD_ALIGN * NPAD_ALIGN;
    if (band > 0) L.n_pad = (n + L.W - 1) / L.W * L.W;
    L.nb = band > 0 ? L.n_pad / L.W : 0;
    L.ld = L.n_pad;
    L.dev_block = dev_block > 0 ? (dev_block + TILE_N - 1) / TILE_N * TILE_N : DEFAULT_DEV_BLOCK;
    L.npb_max = L.n_pad / (precision == GWAS_INT8_SLICED ? trmm_sliced_shape(0).part_rows : MIN_PART_ROWS);
    L.Q = (precision == GWAS_FP64) ? L.Qc + 1 : 1;
    const size_t nn = (size_t)L.ld * (size_t)L.n_pad;
    const size_t A = 256;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes, A); return r; };
    if (band > 0) {
        // per block row U_ii and Gt_i (W x W each); L_ii and E_i of the
        // block row being factored
        L.off_Ub = take((size_t)L.n_pad * L.W * 8);
        L.off_Gt = take((size_t)L.n_pad * L.W * 8);
        L.off_Ab = take((size_t)L.W * L.W * 8);
        L.off_Eb = take((size_t)L.W * L.W * 8);
    } else {
        L.off_L = take(nn * 8);
        L.off_U = take(nn * 8);
    }
    L.off_Ulow = (precision == GWAS_FP32_REFINE) ? take(nn * 4)
               : (precision == GWAS_BF16_REFINE) ? take(nn * 2)
               : (precision == GWAS_BF16X3_REFINE) ? take(nn * 2 * 3)
               : (precision == GWAS_INT8_SLICED) ? take(nn * (size_t)slices) : 0;
    L.off_rscale = (precision == GWAS_INT8_SLICED) ? take((size_t)L.n_pad * 8) : 0;
    L.off_rsum = (precision == GWAS_INT8_SLICED) ? take((size_t)L.n_pad * SLICE_PAIRS_MAX * 4) : 0;
    L.off_XY = take((size_t)L.n_pad * L.Qc * 8);
    L.off_C = take((size_t)L.n_pad * L.Qc * 8);
    L.off_W = (precision != GWAS_FP64) ? take((size_t)L.n_pad * L.Qc * 8) : 0;
    L.off_S = take((size_t)L.q1 * L.Qc * 8);
    L.off_consts = take((size_t)consts_len(L.q1, t) * 8);
    L.off_flags = take(256);
    // room for the schedule and partial sums of every tile shape
    const int at = atype_of(precision);
    const int xd = x_dtype == GWAS_X_I8 ? X_I8 : X_F64;     // the dosages as handed over
    const int xt = prod_xt_of(precision, x_dtype);          // the product's dosage operand
    // the reverse pass runs the float64 product with its default shape
    L.sched_len = band > 0 ? 1 : (size_t)trmm_schedule_len(L.n_pad, L.dev_block,
                                            trmm_geom(A_F64, xd, trmm_default_cfg(A_F64, xd), 0));
    // every admissible shape with the model's and every candidate row group
    for (int c = 0; c < trmm_cfg_limit() && band == 0; ++c) {
        if (!trmm_cfg_valid(at, xt, c)) continue;
        for (int r : {0, 1, 2, 4, 8}) {
            const TrmmShape sh = trmm_geom(at, xt, c, slices, r);
            L.sched_len = std::max(L.sched_len, (size_t)trmm_schedule_len(L.n_pad, L.dev_block, sh));
        }
    }
    L.off_sched = take(L.sched_len * 2 * 4);
    L.off_sched_tail = take(L.sched_len * 2 * 4);
    // the widest multiple of 128 columns (at most dev_block) whose scratch
    // fits the static buffer, and room for its schedule in every shape
    {
        int64_t lo = 0, hi = L.dev_block / TILE_N;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            size_t off[6];
            noalloc_offsets(L, mid * TILE_N, off);
            if (off[5] <= NOALLOC_SCRATCH_BYTES) lo = mid; else hi = mid - 1;
        }
        L.na_cols = band > 0 ? 0 : lo * TILE_N;   // the banded path has no schedule-driven product
        L.na_sched_len = 0;
        if (L.na_cols > 0)
            for (int c = 0; c < trmm_cfg_limit(); ++c) {
                if (!trmm_cfg_valid(at, xt, c)) continue;
                for (int r : {0, 1, 2, 4, 8})
                    L.na_sched_len = std::max(L.na_sched_len, (size_t)trmm_schedule_len(
                                                                  L.n_pad, L.na_cols, trmm_geom(at, xt, c, slices, r)));
            }
        L.off_sched_na = take(std::max<size_t>(L.na_sched_len, 1) * 2 * 4);
    }
    // region shared by the set-up temporary and the streaming buffers
    L.off_region = o;
    const size_t elem = (x_dtype == GWAS_X_I8) ? 1 : 8;
    size_t r = 0;
    auto rtake = [&](size_t bytes) { size_t q = r; r = align_up(r + bytes, A); return L.off_region + q; };
    L.off_xbuf[0] = rtake((size_t)L.n_pad * L.dev_block * elem);
    L.off_xbuf[1] = rtake((size_t)L.n_pad * L.dev_block * elem);
    L.off_part = rtake((size_t)L.npb_max * L.Q * L.dev_block * 8);
    L.off_red = rtake((size_t)chunks_of(L.npb_max) * L.Q * L.dev_block * 8);
    L.off_xw = (precision != GWAS_FP64) ? rtake((size_t)L.Qc * L.dev_block * 8) : 0;
    L.off_xwpart = (precision != GWAS_FP64) ? rtake((size_t)xw_splits(n) * L.Qc * L.dev_block * 8) : 0;
    // float64 dosages cut into bfloat16 (three slices, or one rounding)
    L.off_xsl = x_cut(xt) ? rtake((size_t)x_cut_ld(xt, L.n_pad) * L.dev_block * x_elem_bytes(xt)) : 0;
    for (int s = 0; s < 2; ++s) {
        L.off_b[s] = rtake((size_t)p * t * L.dev_block * 8);
        L.off_v[s] = rtake((size_t)L.dev_block * 8);
        L.off_i[s] = rtake((size_t)L.dev_block * 4);
    }
    // banded: Z of the previous and the current block row
    for (int s = 0; s < 2 && band > 0; ++s) L.off_Z[s] = rtake((size_t)L.W * L.dev_block * 8);
    // the factorisation's temporary (the order it recurses on: n_pad, or W)
    const int64_t nf = band > 0 ? L.W : L.n_pad;
    const int64_t n1 = (nf / 2 + LEAF - 1) / LEAF * LEAF;
    const size_t tmp = (size_t)n1 * (size_t)(nf - n1) * 8;
    L.off_tmp = L.off_region;
    // banded M handed over in host memory: a device copy of its band storage
    // (ldm x n doubles) beside the temporary, for the set-up only
    L.off_bandcopy = L.off_region + align_up(tmp, A);
    const size_t init_bytes = align_up(tmp, A) + (band > 0 ? align_up((size_t)L.band_ld * n * 8, A) : 0);
    L.total = L.off_region + std::max(r, init_bytes);
    return L;
}

}  // namespace

// Serial number of each context, never reused in a process: grouped-launch
// state (schedules, captured graphs) is keyed by these, not by addresses a
// freed context's successor could take over.
static std::atomic<uint64_t> next_ctx_id{1};

struct gwas_ctx {
    uint64_t magic = CTX_MAGIC;
    uint64_t id = next_ctx_id.fetch_add(1);
    uint64_t gen = 0;             // bumped whenever the tile shape or schedule grouping changes
    bool poisoned = false;
    int64_t inject_at = 0;        // test hook: the inject_at-th checked HIP status fails (0 = off)
    bool injected = false;
    // staging slots of the streamed sub-blocks, alternating across calls: a
    // slot reused waits for the events of its previous use
    uint64_t seq = 0;
    bool slot_used[2] = {false, false};
    bool out_used[2] = {false, false};
    // pinned host buffers that pageable dosage blocks are packed into before
    // their copy to the device (allocated at the first pageable block)
    char* pin[2] = {nullptr, nullptr};
    bool pin_used[2] = {false, false};
    bool pin_failed = false;
    int64_t pending = 0;          // blocks queued by gwas_stream_block_async, not yet waited for
    int device = 0;
    Layout lay{};
    char* ws = nullptr;
    bool own_ws = false;
    double *L = nullptr, *U = nullptr, *XY = nullptr, *C = nullptr, *W = nullptr, *S = nullptr,
           *consts = nullptr;
    void* Ulow = nullptr;
    double* rscale = nullptr;
    int* rsum = nullptr;
    double *Ub = nullptr, *Gt = nullptr, *Ab = nullptr, *Eb = nullptr, *Zb[2] = {nullptr, nullptr};   // banded M
    TrmmShape shape{};
    int* flags = nullptr;
    int* sched = nullptr;
    int* sched_tail = nullptr;
    int64_t tail_cols = -1;
    int* sched_na = nullptr;        // schedule of gwas_stream_block_noalloc's sub-blocks
    char* nscratch = nullptr;       // device address of this device's static scratch
    hipEvent_t ev_na = nullptr;     // orders gwas_stream_block_noalloc after queued work
    hipEvent_t ev_fork = nullptr;   // grouped calls: the product is done, per-SNP work may start
    hipEvent_t ev_join = nullptr;   // grouped calls: this context's per-SNP work is done
    int at = A_F64;
    int cfg = 0;
    bool band_walk = false;         // banded M: all block rows of a sub-block in one launch
    int64_t sub = 0;                // sub-block width of gwas_stream_block (dev_block, or the autotuner's)
    int rgroup = 0;                 // schedule row group (0: the traffic model's choice)
    char* xbuf[2] = {nullptr, nullptr};
    double* part = nullptr;
    double* red = nullptr;          // chunk totals of part
    double* xw = nullptr;
    double* xwpart = nullptr;       // split-K partial sums of xw
    __bf16* xsl = nullptr;          // the sub-block's float64 dosages cut into bfloat16 (X_BF16S, X_BF16)
    double* bbuf[2] = {nullptr, nullptr};
    double* vbuf[2] = {nullptr, nullptr};
    int* ibuf[2] = {nullptr, nullptr};
    double* tmp = nullptr;
    hipStream_t s_comp = nullptr, s_h2d = nullptr, s_d2h = nullptr;
    hipStream_t s_user = nullptr;   // caller's stream: joined before each call reads inputs
    hipEvent_t ev_user = nullptr;
    bool own_comp = false;
    hipEvent_t ev_loaded[2] = {}, ev_done[2] = {}, ev_out[2] = {};
    std::vector<int> host_sched, host_tail;
    bool timing = false;
    std::vector<hipEvent_t> tev;    // event pairs around timed launches
    std::vector<int64_t> tcols;     // columns of each timed launch not yet read back
    int64_t t_launches = 0, t_cols = 0;
    double t_ms = 0.0;
    int64_t info = 0;
    std::string err;
    struct Group* grp = nullptr;    // grouped-launch state, owned by the first context of a group
    struct Back* back = nullptr;    // reverse-pass state (gwas_backward_*)
};

// Scratch of gwas_stream_block_noalloc (per-SNP partial sums, chunk totals
// and cross products of one sub-block).  Each device holds its own copy for
// the life of the process; host code uses only the device address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch).
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_addr[MAX_DEVICES] = {};

// Device address of `scratch` on device `dev`, which must be current; looked
// up once per device.
int noalloc_scratch(int dev, char** out) {
    if (dev < 0 || dev >= MAX_DEVICES) return GWAS_E_NO_DEVICE;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return GWAS_E_HIP;
        }
        scratch_addr[dev] = ptr;
    }
    *out = static_cast<char*>(scratch_addr[dev]);
    return GWAS_OK;
}
}  // namespace

// Reverse-pass state: M^-1 = U U^T, W = M^-1 [X_L | y], the constants
// W_L^T W_L and W_L^T w_y, per-sub-block scratch and the accumulators.
struct Back {
    char* mem = nullptr;
    double *Minv = nullptr, *W = nullptr, *GW = nullptr, *part = nullptr, *red = nullptr, *xw = nullptr,
           *contrib = nullptr, *coef = nullptr, *g = nullptr, *acc = nullptr, *v = nullptr,
           *gy = nullptr, *sb = nullptr, *sv = nullptr, *sgb = nullptr, *sgv = nullptr;
    int* si = nullptr;
    int64_t npb = 0;
    bool ready = false;
};

// State of grouped launches (gwas_stream_group), kept by the group's first
// context: the combined tile schedule, per-context kernel arguments (pinned
// host and device copies, double buffered) and an optional captured graph.
struct Group {
    std::vector<uint64_t> key;      // (id, generation) of the contexts the schedule was built for
    int64_t sched_cols = -1;
    int* d_sched = nullptr;
    size_t sched_cap = 0;
    int64_t n_sched = 0;
    TrmmArgs* h_args[2] = {nullptr, nullptr};
    TrmmArgs* d_args[2] = {nullptr, nullptr};
    std::vector<int> host_sched;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> graph_key;  // (id, generation) of the contexts the graph was captured for
    // the graph's own argument array and schedule, never rewritten after capture
    TrmmArgs* h_args_graph = nullptr;
    TrmmArgs* d_args_graph = nullptr;
    int* d_sched_graph = nullptr;
    // float64 groups read device dosages in place in graph mode: the dosage
    // pointers the graph's argument array holds, and pinned copies of the
    // array (alternating) that new pointers are uploaded from
    std::vector<const void*> graph_x;
    std::vector<int64_t> graph_ldx;
    TrmmArgs* h_args_upd[2] = {nullptr, nullptr};
};

namespace {

// Waits for the work a failed call left queued on the context's streams, so
// that no copy into a caller's buffer is still running when the call
// returns.  A stream that is being captured is left alone (the capture ends
// with an error of its own).
void drain(gwas_ctx* c) {
    const hipStream_t ss[3] = {c->s_comp, c->s_h2d, c->s_d2h};
    for (hipStream_t st : ss) {
        if (!st) continue;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
            (void)hipStreamSynchronize(st);
    }
    (void)hipGetLastError();
}

int fail_hip(gwas_ctx* c, hipError_t e, const char* what) {
    if (c) {
        c->err = std::string(what) + ": " + hipGetErrorString(e) + (c->injected ? " (injected)" : "");
        c->poisoned = true;
        drain(c);
    }
    return (e == hipErrorOutOfMemory) ? GWAS_E_OOM : GWAS_E_HIP;
}

// Releases a device object and forgets it before its status is checked, so
// an object is never released twice, whatever the check reports.
template <typename T, typename F> hipError_t drop(T*& p, F release_fn) {
    if (!p) return hipSuccess;
    const hipError_t e = release_fn(p);
    p = nullptr;
    return e;
}

// the fault-injection test hook counts every checked HIP status
bool inject_now(gwas_ctx* c) {
    if (!c || c->inject_at <= 0 || --c->inject_at > 0) return false;
    c->injected = true;
    return true;
}

#define HIPCHK(ctx, expr)                                                         \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ == hipSuccess && inject_now(ctx)) e_ = hipErrorUnknown;            \
        if (e_ != hipSuccess) return fail_hip((ctx), e_, #expr);                  \
    } while (0)

bool live(const gwas_ctx* c) { return c && c->magic == CTX_MAGIC && !c->poisoned; }

// Kernel timing: an event pair around each timed launch, read back once the
// stream has drained (after a synchronous call, or when queued blocks are
// waited for).
int timer_start(gwas_ctx* c, hipStream_t s) {
    const size_t k = c->tcols.size();
    while (c->tev.size() < 2 * (k + 1)) {
        hipEvent_t ev;
        HIPCHK(c, hipEventCreate(&ev));
        c->tev.push_back(ev);
    }
    HIPCHK(c, hipEventRecord(c->tev[2 * k], s));
    return GWAS_OK;
}

int timer_stop(gwas_ctx* c, hipStream_t s, int64_t cols) {
    HIPCHK(c, hipEventRecord(c->tev[2 * c->tcols.size() + 1], s));
    c->tcols.push_back(cols);
    return GWAS_OK;
}

int collect_timing(gwas_ctx* c) {
    for (size_t k = 0; k < c->tcols.size(); ++k) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->tev[2 * k], c->tev[2 * k + 1]));
        c->t_ms += ms;
        c->t_launches += 1;
        c->t_cols += c->tcols[k];
    }
    c->tcols.clear();
    return GWAS_OK;
}

// The caller's current device is restored when an entry point returns.
struct DeviceScope {
    int prev = -1;
    DeviceScope() {
        if (hipGetDevice(&prev) != hipSuccess) {
            (void)hipGetLastError();
            prev = -1;
        }
    }
    ~DeviceScope() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// make `s` wait for everything the caller queued on its own stream so far
hipError_t join_user(gwas_ctx* c, hipStream_t s) {
    hipError_t e = hipEventRecord(c->ev_user, c->s_user);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, c->ev_user, 0);
    return e;
}

bool pinned_host(const void* p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeHost;
}

// The pinned buffers pageable blocks are staged through; false (and the
// runtime's own staging is used) when they cannot be had.
bool ensure_pinned_ring(gwas_ctx* c) {
    if (c->pin[0]) return true;
    if (c->pin_failed) return false;
    const size_t bytes = (size_t)c->lay.n * (size_t)c->lay.dev_block * (c->lay.x_dtype == GWAS_X_I8 ? 1 : 8);
    for (int s = 0; s < 2; ++s) {
        void* ptr = nullptr;
        if (hipHostMalloc(&ptr, bytes, 0) != hipSuccess) {
            (void)hipGetLastError();
            for (int q = 0; q < 2; ++q)
                if (c->pin[q]) (void)hipHostFree(c->pin[q]);
            c->pin[0] = c->pin[1] = nullptr;
            c->pin_failed = true;
            return false;
        }
        c->pin[s] = static_cast<char*>(ptr);
    }
    return true;
}

// cols columns of `bytes` bytes at a stride of `ld` bytes, packed into dst;
// large copies are split over host threads.
void pack_columns(char* dst, const char* src, size_t ld, size_t bytes, int64_t cols) {
    auto work = [=](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c) memcpy(dst + (size_t)c * bytes, src + (size_t)c * ld, bytes);
    };
    const unsigned hw = std::thread::hardware_concurrency();
    const int T = (bytes * (size_t)cols >= (size_t(64) << 20)) ? (int)std::min<unsigned>(8, std::max(1u, hw)) : 1;
    if (T <= 1 || cols < T) {
        work(0, cols);
        return;
    }
    std::vector<std::thread> th;
    int64_t done = 0;   // columns handed to threads that started
    try {
        for (int i = 0; i < T; ++i) {
            th.emplace_back(work, cols * i / T, cols * (i + 1) / T);
            done = cols * (i + 1) / T;
        }
    } catch (...) {
    }
    for (auto& t : th) t.join();
    if (done < cols) work(done, cols);
}

bool on_device(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

// Recursive Cholesky and triangular inverse of the diagonal block [o, o+sz):
//   [A11 .; A21 A22] = [L11 0; L21 L22] [L11 0; L21 L22]^T,
//   L21 = A21 L11^-T, A22 <- A22 - L21 L21^T, and
//   U = L^-T with U12 = -U11 L21^T U22.
// Lm and Um are the factor and its inverse transpose (leading dimension ld);
// element 0 is row `row0` of M, for the failing-pivot report.
int chol_inv(gwas_ctx* c, double* Lm, double* Um, int64_t ld, int64_t row0, int64_t o, int64_t sz) {
    hipStream_t s = c->s_comp;
    if (sz == LEAF) {
        HIPCHK(c, chol_leaf(Lm + o + o * ld, Um + o + o * ld, ld, row0 + o, c->lay.n, c->flags, s));
        return GWAS_OK;
    }
    const int64_t n1 = (sz / 2 + LEAF - 1) / LEAF * LEAF;
    const int64_t n2 = sz - n1;
    int rc = chol_inv(c, Lm, Um, ld, row0, o, n1);
    if (rc) return rc;
    double* L21 = Lm + (o + n1) + o * ld;
    double* L22 = Lm + (o + n1) + (o + n1) * ld;
    double* U11 = Um + o + o * ld;
    double* U12 = Um + o + (o + n1) * ld;
    double* U22 = Um + (o + n1) + (o + n1) * ld;
    // T = A21 U11 (= L21), copied into place
    GemmArgs g{};
    g = GemmArgs{n2, n1, n1, L21, ld, 'N', U11, ld, 'N', c->tmp, n2, 1.0, 0.0, KR_B_UPPER, 0};
    HIPCHK(c, gemm_f64(g, s));
    HIPCHK(c, hipMemcpy2DAsync(L21, ld * 8, c->tmp, n2 * 8, n2 * 8, n1, hipMemcpyDeviceToDevice, s));
    // A22 -= L21 L21^T (lower tiles)
    g = GemmArgs{n2, n2, n1, c->tmp, n2, 'N', c->tmp, n2, 'T', L22, ld, -1.0, 1.0, 0, 1};
    HIPCHK(c, gemm_f64(g, s));
    rc = chol_inv(c, Lm, Um, ld, row0, o + n1, n2);
    if (rc) return rc;
    // T = U11 L21^T (n1 x n2), U12 = -T U22
    g = GemmArgs{n1, n2, n1, U11, ld, 'N', L21, ld, 'T', c->tmp, n1, 1.0, 0.0, KR_A_UPPER, 0};
    HIPCHK(c, gemm_f64(g, s));
    g = GemmArgs{n1, n2, n2, c->tmp, n1, 'N', U22, ld, 'N', U12, ld, -1.0, 0.0, KR_B_UPPER, 0};
    HIPCHK(c, gemm_f64(g, s));
    return GWAS_OK;
}

int check_device(int dev, std::string& why) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        why = "no HIP device";
        return GWAS_E_NO_DEVICE;
    }
    if (dev < 0 || dev >= count) {
        why = "device ordinal out of range";
        return GWAS_E_NO_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        why = "hipGetDeviceProperties failed";
        return GWAS_E_NO_DEVICE;
    }
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        why = std::string("device is ") + prop.gcnArchName + ", the library is built for gfx950";
        return GWAS_E_NO_DEVICE;
    }
    return GWAS_OK;
}

void release(gwas_ctx* c) {
    if (!c) return;
    if (c->s_comp) (void)hipStreamSynchronize(c->s_comp);
    if (c->s_h2d) (void)hipStreamSynchronize(c->s_h2d);
    if (c->s_d2h) (void)hipStreamSynchronize(c->s_d2h);
    for (int s = 0; s < 2; ++s) {
        if (c->ev_loaded[s]) (void)hipEventDestroy(c->ev_loaded[s]);
        if (c->ev_done[s]) (void)hipEventDestroy(c->ev_done[s]);
        if (c->ev_out[s]) (void)hipEventDestroy(c->ev_out[s]);
    }
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    if (c->back) {
        if (c->back->mem) (void)hipFree(c->back->mem);
        delete c->back;
        c->back = nullptr;
    }
    if (c->grp) {
        Group* g = c->grp;
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        for (int s = 0; s < 2; ++s) {
            if (g->h_args[s]) (void)hipHostFree(g->h_args[s]);
            if (g->d_args[s]) (void)hipFree(g->d_args[s]);
        }
        if (g->d_sched) (void)hipFree(g->d_sched);
        if (g->h_args_graph) (void)hipHostFree(g->h_args_graph);
        for (int s = 0; s < 2; ++s)
            if (g->h_args_upd[s]) (void)hipHostFree(g->h_args_upd[s]);
        if (g->d_args_graph) (void)hipFree(g->d_args_graph);
        if (g->d_sched_graph) (void)hipFree(g->d_sched_graph);
        delete g;
        c->grp = nullptr;
    }
    if (c->s_h2d) (void)hipStreamDestroy(c->s_h2d);
    if (c->s_d2h) (void)hipStreamDestroy(c->s_d2h);
    if (c->own_comp && c->s_comp) (void)hipStreamDestroy(c->s_comp);
    if (c->ev_user) (void)hipEventDestroy(c->ev_user);
    if (c->ev_na) (void)hipEventDestroy(c->ev_na);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    for (int s = 0; s < 2; ++s)
        if (c->pin[s]) (void)hipHostFree(c->pin[s]);
    (void)hipGetLastError();
}

int upload_schedule(gwas_ctx* c, int64_t cols, int* dst, std::vector<int>& host) {
    const TrmmShape sh = c->shape;
    const int64_t len = trmm_schedule_len(c->lay.n_pad, cols, sh);
    host.assign((size_t)(2 * len), 0);
    if (len > (int64_t)c->lay.sched_len ||
        trmm_schedule(c->lay.n_pad, cols, sh, host.data(), len) != len) {
        c->err = "tile schedule does not fit";
        return GWAS_E_INVALID;
    }
    HIPCHK(c, hipMemcpyAsync(dst, host.data(), host.size() * sizeof(int), hipMemcpyHostToDevice,
                             c->s_comp));
    return GWAS_OK;
}

// Schedule of gwas_stream_block_noalloc's sub-blocks (na_cols columns; the
// last sub-block of a call may be narrower and runs the same schedule).
int upload_noalloc_schedule(gwas_ctx* c) {
    const Layout& Y = c->lay;
    if (Y.na_cols <= 0) return GWAS_OK;
    const int64_t len = trmm_schedule_len(Y.n_pad, Y.na_cols, c->shape);
    std::vector<int> host((size_t)(2 * len), 0);
    if (len > (int64_t)Y.na_sched_len || trmm_schedule(Y.n_pad, Y.na_cols, c->shape, host.data(), len) != len) {
        c->err = "tile schedule does not fit";
        return GWAS_E_INVALID;
    }
    // synchronous: the host vector is released on return
    HIPCHK(c, hipMemcpy(c->sched_na, host.data(), host.size() * sizeof(int), hipMemcpyHostToDevice));
    return GWAS_OK;
}

// xs: where the sub-block's cut dosages are (X_BF16S, X_BF16; NULL: the
// context's own buffer)
TrmmArgs trmm_args_for(const gwas_ctx* c, const void* xptr, int64_t xld, int64_t cols,
                       const __bf16* xs = nullptr) {
    const Layout& Y = c->lay;
    TrmmArgs ta{};
    ta.at = c->at;
    ta.xt = prod_xt_of(Y.precision, Y.x_dtype);
    ta.cfg = c->cfg;
    ta.slices = Y.slices;
    ta.rscale = c->rscale;
    ta.rsum = c->rsum;
    ta.Ut = (c->at == A_F64) ? (const void*)c->U : c->Ulow;
    ta.ldu = (Y.precision == GWAS_BF16X3_REFINE) ? 3 * Y.n_pad : Y.ld;   // slices one after another
    ta.n_pad = Y.n_pad;
    ta.X = xptr;
    ta.ldx = xld;
    ta.Xd = xptr;
    ta.ldxd = xld;
    if (x_cut(ta.xt)) {
        ta.X = xs ? xs : c->xsl;
        ta.ldx = x_cut_ld(ta.xt, Y.n_pad);
    }
    ta.n = Y.n;
    ta.cols = cols;
    ta.C = c->C;
    ta.ldc = Y.n_pad;
    ta.Qc = Y.Qc;
    ta.with_cross = (Y.precision == GWAS_FP64);
    ta.part = c->part;
    ta.ldp = Y.dev_block;
    ta.sched = c->sched;
    ta.rgroup = c->rgroup;
    ta.n_sched = trmm_schedule_len(Y.n_pad, cols, c->shape);
    return ta;
}

// Float64 dosages of the bfloat16 products are cut into bfloat16 once per
// sub-block, before its product (into out: three slices, 3 n_pad per column,
// for the bfloat16-slice mode; one rounding, n_pad per column, for the
// bfloat16 mode); other modes have nothing to do.  xargs: read the dosages'
// address from a device argument record when the kernel runs (replayed
// graphs).
hipError_t cut_dosages(const gwas_ctx* c, const void* xptr, int64_t xld, int64_t cols, __bf16* out, hipStream_t s,
                       const TrmmArgs* xargs = nullptr) {
    const Layout& Y = c->lay;
    const int xt = prod_xt_of(Y.precision, Y.x_dtype);
    const double* X = static_cast<const double*>(xptr);
    if (xt == X_BF16S) return slice_x_bf16(X, xld, Y.n, Y.n_pad, cols, out, 3 * Y.n_pad, s, xargs);
    if (xt == X_BF16) return convert_x_bf16(X, xld, Y.n, Y.n_pad, cols, out, Y.n_pad, s, xargs);
    return hipSuccess;
}

// Device scratch of the per-SNP stage of one sub-block: the product's
// partial sums, their chunk totals and (reduced modes) the cross products
// x^T W with their split-K partials, all with leading dimension ld (>= the
// sub-block's columns).
struct SubScratch {
    double* part;
    double* red;
    double* xw;
    double* xwpart;
    int64_t ld;
};

SubScratch ctx_scratch(const gwas_ctx* c) {
    return SubScratch{c->part, c->red, c->xw, c->xwpart, c->lay.dev_block};
}

SolveArgs solve_args_for(const gwas_ctx* c, const SubScratch& sc, int64_t cols, double* bo, int64_t ldbo,
                         double* vo, int* io) {
    const Layout& Y = c->lay;
    SolveArgs sa{};
    sa.p = Y.p;
    sa.t = Y.t;
    sa.cols = cols;
    sa.part = sc.red;   // chunk totals of the partial sums
    sa.ldp = sc.ld;
    sa.npb = chunks_of(Y.n_pad / c->shape.part_rows);
    sa.Q = Y.Q;
    sa.xw = sc.xw;
    sa.ldxw = sc.ld;
    sa.consts = c->consts;
    sa.refine = (Y.precision == GWAS_FP64) ? 0 : REFINE_STEPS;
    sa.rank_tol = (Y.precision == GWAS_FP64) ? RANK_TOL_F64
                : (Y.precision == GWAS_FP32_REFINE) ? RANK_TOL_F32
                : (Y.precision == GWAS_BF16_REFINE) ? RANK_TOL_BF16
                : (Y.precision == GWAS_BF16X3_REFINE) ? RANK_TOL_F32 : RANK_TOL_I8S;
    sa.b = bo;
    sa.ldb = ldbo;
    sa.var = vo;
    sa.info = io;
    return sa;
}

// Cross products x^T W (reduced modes) and the per-SNP solves of one sub-block.
hipError_t finish_sub(const gwas_ctx* c, const SubScratch& sc, const void* xptr, int64_t xld, int64_t cols,
                      double* bo, int64_t ldbo, double* vo, int* io, hipStream_t s,
                      const TrmmArgs* xargs = nullptr) {
    const Layout& Y = c->lay;
    if (Y.precision != GWAS_FP64) {
        // the paired-digit int8 product is exact only for dosages 0, 1, 2:
        // other values turn the SNP's results into NaN
        const bool check012 = Y.precision == GWAS_INT8_SLICED && trmm_sliced_paired(c->cfg);
        hipError_t e = snp_cross_w((Y.x_dtype == GWAS_X_I8) ? X_I8 : X_F64, xptr, xld, Y.n, cols, c->W,
                                   Y.n_pad, Y.Qc, sc.xw, sc.ld, sc.xwpart,
                                   (int64_t)xw_splits(Y.n) * Y.Qc * sc.ld, s, check012, xargs);
        if (e != hipSuccess) return e;
    }
    hipError_t e = partial_chunks(sc.part, sc.ld, Y.n_pad / c->shape.part_rows, (int)Y.Q, cols,
                                  PART_CHUNK, sc.red, sc.ld, s);
    if (e != hipSuccess) return e;
    return snp_solve(solve_args_for(c, sc, cols, bo, ldbo, vo, io), s);
}

// Combined tile schedule of several contexts with one tile shape: every
// (context, row block) is a unit of work (K length x column tiles), dealt
// longest first to the least loaded of the 8 XCD lists (workgroup b runs on
// XCD b % 8); each list keeps its units in that order.
int64_t group_schedule(const std::vector<gwas_ctx*>& cs, int64_t cols, std::vector<int>& out) {
    std::vector<int64_t> nrb(cs.size());
    for (size_t c = 0; c < cs.size(); ++c) nrb[c] = cs[c]->lay.n_pad / cs[0]->shape.tm;
    return trmm_schedule_multi(nrb.data(), (int)cs.size(), cols, cs[0]->shape, &out);
}

// Set-up for a banded M (half-bandwidth w, blocks of W rows): block row by
// block row, A_ii = M_ii - E_i E_i^T = L_ii L_ii^T (with U_ii = L_ii^-T),
// Gt_i = -E_i^T U_ii and E_{i+1} = M_{i+1,i} U_ii; then the whitened
// C = L^-1 [X_L | Y] by the same block forward substitution the streamed
// blocks take, C_i = U_ii^T XY_i + Gt_i^T C_{i-1}.
int init_banded(gwas_ctx* c, const gwas_desc* d) {
    const Layout& Y = c->lay;
    const int64_t n = Y.n, n_pad = Y.n_pad, W = Y.W, w = Y.band;
    hipStream_t s = c->s_comp;
    const double* AB = d->M;
    if (!d->inputs_on_device) {
        double* cp = reinterpret_cast<double*>(c->ws + Y.off_bandcopy);
        HIPCHK(c, hipMemcpyAsync(cp, d->M, (size_t)d->ldm * n * 8, hipMemcpyHostToDevice, s));
        AB = cp;
    }
    HIPCHK(c, hipMemsetAsync(c->Ub, 0, (size_t)n_pad * W * 8, s));
    for (int64_t i = 0; i < Y.nb; ++i) {
        double* Ui = c->Ub + i * W * W;
        double* Gi = c->Gt + i * W * W;
        HIPCHK(c, band_block(AB, d->ldm, w, n, i * W, i * W, W, W, c->Ab, W, s));
        GemmArgs g{};
        if (i > 0) {
            g = GemmArgs{W, W, W, c->Eb, W, 'N', c->Eb, W, 'T', c->Ab, W, -1.0, 1.0, 0, 1};
            HIPCHK(c, gemm_f64(g, s));
        }
        int rc = chol_inv(c, c->Ab, Ui, W, i * W, 0, W);
        if (rc) return rc;
        if (i > 0) {
            g = GemmArgs{W, W, W, c->Eb, W, 'T', Ui, W, 'N', Gi, W, -1.0, 0.0, KR_B_UPPER, 0};
            HIPCHK(c, gemm_f64(g, s));
        }
        if (i + 1 < Y.nb) {
            HIPCHK(c, band_block(AB, d->ldm, w, n, (i + 1) * W, i * W, W, W, c->Ab, W, s));
            g = GemmArgs{W, W, W, c->Ab, W, 'N', Ui, W, 'N', c->Eb, W, 1.0, 0.0, KR_B_UPPER, 0};
            HIPCHK(c, gemm_f64(g, s));
        }
    }
    const hipMemcpyKind kin = d->inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(c, hipMemsetAsync(c->XY, 0, (size_t)n_pad * Y.Qc * 8, s));
    HIPCHK(c, hipMemcpy2DAsync(c->XY, n_pad * 8, d->XL, d->ldxl * 8, n * 8, Y.q1, kin, s));
    HIPCHK(c, hipMemcpy2DAsync(c->XY + (size_t)n_pad * Y.q1, n_pad * 8, d->Y, d->ldy * 8, n * 8, Y.t, kin, s));
    for (int64_t i = 0; i < Y.nb; ++i) {
        GemmArgs g{W, Y.Qc, W, c->Ub + i * W * W, W, 'T', c->XY + i * W, n_pad, 'N', c->C + i * W, n_pad,
                   1.0, 0.0, KR_A_LOWER, 0};
        HIPCHK(c, gemm_f64(g, s));
        if (i > 0) {
            g = GemmArgs{W, Y.Qc, W, c->Gt + i * W * W, W, 'T', c->C + (i - 1) * W, n_pad, 'N', c->C + i * W,
                         n_pad, 1.0, 1.0, 0, 0};
            HIPCHK(c, gemm_f64(g, s));
        }
    }
    return GWAS_OK;
}

int init_body(gwas_ctx* c, const gwas_desc* d) {
    const Layout& Y = c->lay;
    const int64_t ld = Y.ld, n = Y.n, n_pad = Y.n_pad;
    hipStream_t s = c->s_comp;
    const hipMemcpyKind kin = d->inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;

    HIPCHK(c, join_user(c, s));
    HIPCHK(c, hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(c->flags), INT_MAX, 1, s));
    HIPCHK(c, hipMemsetAsync(c->flags + 1, 0, 4, s));
    GemmArgs g{};
    if (Y.band > 0) {
        int rc = init_banded(c, d);
        if (rc) return rc;
    } else {
        // M -> L (the lower triangle is what the factorisation reads), identity padding
        HIPCHK(c, hipMemcpy2DAsync(c->L, ld * 8, d->M, d->ldm * 8, n * 8, n, kin, s));
        HIPCHK(c, pad_identity(c->L, ld, n, n_pad, s));
        HIPCHK(c, hipMemsetAsync(c->U, 0, (size_t)ld * n_pad * 8, s));
        int rc = chol_inv(c, c->L, c->U, ld, 0, 0, n_pad);
        if (rc) return rc;
        // [X_L | Y] with zero padding rows, then C = L^-1 [X_L | Y]
        HIPCHK(c, hipMemsetAsync(c->XY, 0, (size_t)n_pad * Y.Qc * 8, s));
        HIPCHK(c, hipMemcpy2DAsync(c->XY, n_pad * 8, d->XL, d->ldxl * 8, n * 8, Y.q1, kin, s));
        HIPCHK(c, hipMemcpy2DAsync(c->XY + (size_t)n_pad * Y.q1, n_pad * 8, d->Y, d->ldy * 8, n * 8,
                                   Y.t, kin, s));
        g = GemmArgs{n_pad, Y.Qc, n_pad, c->U, ld, 'T', c->XY, n_pad, 'N', c->C, n_pad, 1.0, 0.0,
                     KR_A_LOWER, 0};
        HIPCHK(c, gemm_f64(g, s));
    }
    // [S_TL | bbar_T] = Xbar_L^T [Xbar_L | Ybar]
    g = GemmArgs{Y.q1, Y.Qc, n_pad, c->C, n_pad, 'T', c->C, n_pad, 'N', c->S, Y.q1, 1.0, 0.0, 0, 0};
    HIPCHK(c, gemm_f64(g, s));
    HIPCHK(c, snp_constants(c->S, Y.q1, Y.q1, Y.t, c->consts, c->flags + 1, s));
    if (Y.precision != GWAS_FP64) {
        // W = L^-T [Xbar_L | Ybar] = M^-1 [X_L | Y]
        g = GemmArgs{n_pad, Y.Qc, n_pad, c->U, ld, 'N', c->C, n_pad, 'N', c->W, n_pad, 1.0, 0.0,
                     KR_A_UPPER, 0};
        HIPCHK(c, gemm_f64(g, s));
        if (Y.precision == GWAS_FP32_REFINE)
            HIPCHK(c, convert_f32(c->U, (float*)c->Ulow, ld, n_pad, n_pad, s));
        else if (Y.precision == GWAS_BF16X3_REFINE)
            HIPCHK(c, slice_bf16(c->U, ld, n_pad, (__bf16*)c->Ulow, 3 * n_pad, s));
        else if (Y.precision == GWAS_BF16_REFINE)
            HIPCHK(c, convert_bf16(c->U, (__bf16*)c->Ulow, ld, n_pad, n_pad, s));
        else
            HIPCHK(c, slice_rows(c->U, ld, n_pad, Y.n, Y.slices, (int8_t*)c->Ulow, n_pad, c->rscale, c->rsum, s));
    }
    if (Y.band == 0) {
        c->sub = Y.dev_block;
        int rc = upload_schedule(c, c->sub, c->sched, c->host_sched);
        if (rc) return rc;
        rc = upload_noalloc_schedule(c);
        if (rc) return rc;
    }
    HIPCHK(c, hipStreamSynchronize(s));
    int flags[2] = {0, 0};
    HIPCHK(c, hipMemcpy(flags, c->flags, sizeof(flags), hipMemcpyDeviceToHost));
    if (flags[0] != INT_MAX) {
        c->info = flags[0];
        c->err = "M is not positive definite";
        return GWAS_E_NOT_SPD;
    }
    if (flags[1] != 0) {
        c->info = flags[1];
        c->err = "X_L^T M^-1 X_L is not positive definite";
        return GWAS_E_RANK_XL;
    }
    return GWAS_OK;
}

}  // namespace

extern "C" {

size_t gwas_workspace_bytes(int64_t n, int32_t p, int32_t t, int64_t dev_block, int32_t precision,
                            int32_t x_dtype) {
    if (!sizes_valid(n, p, t, dev_block, precision, x_dtype)) return 0;
    return make_layout(n, p, t, dev_block, precision, x_dtype, DEFAULT_SLICES).total;
}

size_t gwas_workspace_bytes_band(int64_t n, int32_t p, int32_t t, int64_t dev_block, int64_t band, int64_t ldm,
                                 int32_t x_dtype) {
    if (band < 1 || ldm < band + 1 || !sizes_valid(n, p, t, dev_block, GWAS_FP64, x_dtype, band)) return 0;
    return make_layout(n, p, t, dev_block, GWAS_FP64, x_dtype, 0, band, ldm).total;
}

int gwas_init(gwas_ctx** out, const gwas_desc* d) {
    if (!out) return GWAS_E_INVALID;
    *out = nullptr;
    if (!d || !d->M || !d->XL || !d->Y) return GWAS_E_INVALID;
    if (!sizes_valid(d->n, d->p, d->t, d->dev_block, d->precision, d->x_dtype, d->band)) return GWAS_E_INVALID;
    if (d->ldm < (d->band > 0 ? d->band + 1 : d->n) || d->ldxl < d->n || d->ldy < d->n) return GWAS_E_INVALID;
    if (d->workspace && (reinterpret_cast<uintptr_t>(d->workspace) % 256)) return GWAS_E_INVALID;
    const int slices = (d->precision == GWAS_INT8_SLICED) ? (d->slices ? d->slices : DEFAULT_SLICES) : 0;
    if (d->precision == GWAS_INT8_SLICED && (slices < 4 || slices > 6)) return GWAS_E_INVALID;

    gwas_ctx* c = new (std::nothrow) gwas_ctx();
    if (!c) return GWAS_E_OOM;
    c->device = d->device;
    std::string why;
    int rc = check_device(d->device, why);
    if (rc) {
        delete c;
        return rc;
    }
    c->lay = make_layout(d->n, d->p, d->t, d->dev_block, d->precision, d->x_dtype, slices, d->band, d->ldm);
    const Layout& Y = c->lay;
    c->at = atype_of(d->precision);
    const int pxt = prod_xt_of(d->precision, d->x_dtype);
    c->cfg = trmm_default_cfg(c->at, pxt);
    if (const char* e = getenv("GWAS_TRMM_CFG")) {
        // tile-shape override for measurement; ignored when not valid here
        const int v = atoi(e);
        if (trmm_cfg_valid(c->at, pxt, v)) c->cfg = v;
    }
    c->shape = trmm_geom(c->at, pxt, c->cfg, slices);
    // the banded product has its own fixed tile (128 x 128, 32-row slices)
    if (d->band > 0) c->shape = TrmmShape{128, 128, band_part_rows(), 512, 1, 32};
    if (d->band > 0) {
        c->band_walk = band_walk_fits(d->x_dtype == GWAS_X_I8 ? X_I8 : X_F64, Y.W);
        // one launch per block row instead, for measurement and tests
        if (const char* e = getenv("GWAS_BAND_STEP")) c->band_walk = c->band_walk && atoi(e) == 0;
    }
    auto bail = [&](int code) {
        release(c);
        c->magic = CTX_DEAD;
        delete c;
        return code;
    };
    DeviceScope scope;
    if (hipSetDevice(d->device) != hipSuccess) return bail(GWAS_E_NO_DEVICE);
    if (int rc2 = noalloc_scratch(d->device, &c->nscratch)) return bail(rc2);
    if (d->workspace) {
        if (d->workspace_bytes < Y.total) return bail(GWAS_E_WORKSPACE);
        c->ws = static_cast<char*>(d->workspace);
    } else {
        if (hipMalloc(&c->ws, Y.total) != hipSuccess) {
            (void)hipGetLastError();
            c->ws = nullptr;
            return bail(GWAS_E_OOM);
        }
        c->own_ws = true;
    }
    char* w = c->ws;
    c->L = (double*)(w + Y.off_L);
    c->U = (double*)(w + Y.off_U);
    c->Ulow = Y.off_Ulow ? (void*)(w + Y.off_Ulow) : nullptr;
    c->rscale = Y.off_rscale ? (double*)(w + Y.off_rscale) : nullptr;
    c->rsum = Y.off_rsum ? (int*)(w + Y.off_rsum) : nullptr;
    c->XY = (double*)(w + Y.off_XY);
    c->C = (double*)(w + Y.off_C);
    c->W = Y.off_W ? (double*)(w + Y.off_W) : nullptr;
    c->S = (double*)(w + Y.off_S);
    c->consts = (double*)(w + Y.off_consts);
    c->flags = (int*)(w + Y.off_flags);
    c->sched = (int*)(w + Y.off_sched);
    c->sched_tail = (int*)(w + Y.off_sched_tail);
    c->sched_na = (int*)(w + Y.off_sched_na);
    for (int s = 0; s < 2; ++s) {
        c->xbuf[s] = w + Y.off_xbuf[s];
        c->bbuf[s] = (double*)(w + Y.off_b[s]);
        c->vbuf[s] = (double*)(w + Y.off_v[s]);
        c->ibuf[s] = (int*)(w + Y.off_i[s]);
    }
    c->part = (double*)(w + Y.off_part);
    c->red = (double*)(w + Y.off_red);
    c->xw = Y.off_xw ? (double*)(w + Y.off_xw) : nullptr;
    c->xwpart = Y.off_xwpart ? (double*)(w + Y.off_xwpart) : nullptr;
    c->xsl = Y.off_xsl ? (__bf16*)(w + Y.off_xsl) : nullptr;
    c->tmp = (double*)(w + Y.off_tmp);
    if (Y.band > 0) {
        c->Ub = (double*)(w + Y.off_Ub);
        c->Gt = (double*)(w + Y.off_Gt);
        c->Ab = (double*)(w + Y.off_Ab);
        c->Eb = (double*)(w + Y.off_Eb);
        for (int s = 0; s < 2; ++s) c->Zb[s] = (double*)(w + Y.off_Z[s]);
        c->L = c->U = nullptr;
    }

    // The library computes on streams of its own (default priority); work the
    // caller queued on its stream before a call is joined through an event.
    c->s_user = static_cast<hipStream_t>(d->stream);
    hipError_t e = hipStreamCreateWithFlags(&c->s_comp, hipStreamNonBlocking);
    c->own_comp = true;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_user, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_na, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->s_h2d, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->s_d2h, hipStreamNonBlocking);
    for (int s = 0; s < 2 && e == hipSuccess; ++s) {
        e = hipEventCreateWithFlags(&c->ev_loaded[s], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_done[s], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_out[s], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return bail(GWAS_E_HIP);
    }
    rc = init_body(c, d);
    if (rc == GWAS_E_NOT_SPD || rc == GWAS_E_RANK_XL) {
        c->poisoned = true;   // info stays readable; streaming is refused
        *out = c;
        return rc;
    }
    if (rc) return bail(rc);
    *out = c;
    return GWAS_OK;
}

namespace {

// Waits for the blocks gwas_stream_block_async queued on the context.
int settle(gwas_ctx* c) {
    if (c->pending == 0) return GWAS_OK;
    HIPCHK(c, hipStreamSynchronize(c->s_h2d));
    HIPCHK(c, hipStreamSynchronize(c->s_comp));
    HIPCHK(c, hipStreamSynchronize(c->s_d2h));
    c->pending = 0;
    return collect_timing(c);
}

// The banded forward substitution of one sub-block: one launch per block
// row, Z alternating between the two buffers; partial sums as the dense
// product's.
hipError_t band_product(const gwas_ctx* c, const void* xptr, int64_t xld, int64_t cols, hipStream_t s) {
    const Layout& Y = c->lay;
    if (c->band_walk) {
        BandArgs ba{};
        ba.xt = X_I8;
        ba.W = Y.W;
        ba.nb = Y.nb;
        ba.Ut = c->Ub;
        ba.Gt = c->Gt;
        ba.X = xptr;
        ba.ldx = xld;
        ba.n = Y.n;
        ba.cols = cols;
        ba.C = c->C;
        ba.ldc = Y.n_pad;
        ba.Qc = Y.Qc;
        ba.part = c->part;
        ba.ldp = Y.dev_block;
        return band_walk(ba, s);
    }
    for (int64_t i = 0; i < Y.nb; ++i) {
        BandArgs ba{};
        ba.xt = (Y.x_dtype == GWAS_X_I8) ? X_I8 : X_F64;
        ba.W = Y.W;
        ba.blk = i;
        ba.Ut = c->Ub + i * Y.W * Y.W;
        ba.Gt = i > 0 ? c->Gt + i * Y.W * Y.W : nullptr;
        ba.X = xptr;
        ba.ldx = xld;
        ba.n = Y.n;
        ba.cols = cols;
        ba.Zprev = i > 0 ? c->Zb[(i - 1) & 1] : nullptr;
        ba.Zcur = c->Zb[i & 1];
        ba.ldz = Y.W;
        ba.C = c->C;
        ba.ldc = Y.n_pad;
        ba.Qc = Y.Qc;
        ba.part = c->part;
        ba.ldp = Y.dev_block;
        const hipError_t e = band_step(ba, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// One pass of Algorithm 2's loop for a block, queued on the context's
// streams without waiting: per sub-block the copy in (when the dosages are
// not read in place), the product, the per-SNP kernels and the copy out (when
// the outputs are not on the device).  Sub-blocks alternate between two
// staging slots across calls, so the next block's copies can run behind this
// block's products.  With `timed`, events bracket each product (launch k uses
// events 2k and 2k+1).
int enqueue_block(gwas_ctx* c, const void* XR, int64_t ldx, int64_t mblk, double* b, int64_t ldb,
                  double* var_snp, int32_t* info, bool timed) {
    const Layout& Y = c->lay;
    HIPCHK(c, join_user(c, c->s_comp));
    HIPCHK(c, hipStreamWaitEvent(c->s_h2d, c->ev_user, 0));
    const size_t elem = (Y.x_dtype == GWAS_X_I8) ? 1 : 8;
    const char* xr = static_cast<const char*>(XR);
    const bool x_dev = on_device(XR);
    const bool direct_x = x_dev && (reinterpret_cast<uintptr_t>(XR) % 16 == 0) &&
                          ((ldx * (int64_t)elem) % 16 == 0) && ldx * (int64_t)elem <= X_DIRECT_MAX_LD_BYTES;
    // pageable host dosages: packed into pinned buffers by the host while the
    // device works on the sub-block before, then copied asynchronously
    const bool stage_host = !x_dev && !pinned_host(XR) && ensure_pinned_ring(c);
    const bool direct_out = on_device(b) && (!var_snp || on_device(var_snp)) &&
                            (!info || on_device(info));
    const int pt = Y.p * Y.t;
    const int64_t sub = c->sub > 0 ? c->sub : Y.dev_block;
    const int64_t nsub = (mblk + sub - 1) / sub;

    for (int64_t k = 0; k < nsub; ++k) {
        const int64_t col0 = k * sub;
        const int64_t cols = std::min<int64_t>(sub, mblk - col0);
        const int slot = (int)(c->seq++ & 1);
        const void* xptr;
        int64_t xld;
        if (direct_x) {
            xptr = xr + (size_t)col0 * ldx * elem;
            xld = ldx;
        } else {
            // the slot's previous sub-block has finished reading it
            if (c->slot_used[slot]) HIPCHK(c, hipStreamWaitEvent(c->s_h2d, c->ev_done[slot], 0));
            const char* src = xr + (size_t)col0 * ldx * elem;
            int64_t sld = ldx * (int64_t)elem;
            if (stage_host) {
                // the pinned slot's last copy to the device has finished
                if (c->pin_used[slot]) HIPCHK(c, hipEventSynchronize(c->ev_loaded[slot]));
                pack_columns(c->pin[slot], src, (size_t)sld, (size_t)Y.n * elem, cols);
                src = c->pin[slot];
                sld = Y.n * (int64_t)elem;
                c->pin_used[slot] = true;
            }
            HIPCHK(c, hipMemcpy2DAsync(c->xbuf[slot], Y.n_pad * elem, src, sld, Y.n * elem, cols,
                                       hipMemcpyDefault, c->s_h2d));
            HIPCHK(c, hipEventRecord(c->ev_loaded[slot], c->s_h2d));
            HIPCHK(c, hipStreamWaitEvent(c->s_comp, c->ev_loaded[slot], 0));
            xptr = c->xbuf[slot];
            xld = Y.n_pad;
        }
        double* bo;
        double* vo;
        int* io;
        int64_t ldbo;
        if (direct_out) {
            bo = b + (size_t)col0 * ldb;
            vo = var_snp ? var_snp + col0 : nullptr;
            io = info ? info + col0 : nullptr;
            ldbo = ldb;
        } else {
            // the slot's previous results have been copied out
            if (c->out_used[slot]) HIPCHK(c, hipStreamWaitEvent(c->s_comp, c->ev_out[slot], 0));
            bo = c->bbuf[slot];
            vo = c->vbuf[slot];
            io = c->ibuf[slot];
            ldbo = pt;
        }
        const int* sched = c->sched;
        if (cols != sub && Y.band == 0) {
            if (cols != c->tail_cols) {
                // the host copy of the tail schedule is rewritten: queued
                // blocks may still be reading it
                if (c->pending) HIPCHK(c, hipStreamSynchronize(c->s_comp));
                int rc = upload_schedule(c, cols, c->sched_tail, c->host_tail);
                if (rc) return rc;
                c->tail_cols = cols;
            }
            sched = c->sched_tail;
        }
        if (timed) {
            if (int rc = timer_start(c, c->s_comp)) return rc;
        }
        if (Y.band > 0) {
            HIPCHK(c, band_product(c, xptr, xld, cols, c->s_comp));
        } else {
            HIPCHK(c, cut_dosages(c, xptr, xld, cols, c->xsl, c->s_comp));
            TrmmArgs ta = trmm_args_for(c, xptr, xld, cols);
            ta.sched = sched;
            HIPCHK(c, trmm_stream(ta, c->s_comp));
        }
        if (timed) {
            if (int rc = timer_stop(c, c->s_comp, cols)) return rc;
        }
        HIPCHK(c, finish_sub(c, ctx_scratch(c), xptr, xld, cols, bo, ldbo, vo, io, c->s_comp));
        HIPCHK(c, hipEventRecord(c->ev_done[slot], c->s_comp));
        c->slot_used[slot] = true;
        if (!direct_out) {
            HIPCHK(c, hipStreamWaitEvent(c->s_d2h, c->ev_done[slot], 0));
            HIPCHK(c, hipMemcpy2DAsync(b + (size_t)col0 * ldb, ldb * 8, bo, pt * 8, pt * 8, cols,
                                       hipMemcpyDefault, c->s_d2h));
            if (var_snp)
                HIPCHK(c, hipMemcpyAsync(var_snp + col0, vo, cols * 8, hipMemcpyDefault, c->s_d2h));
            if (info)
                HIPCHK(c, hipMemcpyAsync(info + col0, io, cols * 4, hipMemcpyDefault, c->s_d2h));
            HIPCHK(c, hipEventRecord(c->ev_out[slot], c->s_d2h));
            c->out_used[slot] = true;
        }
    }
    return GWAS_OK;
}

int check_block_args(const gwas_ctx* c, const void* XR, int64_t ldx, int64_t mblk, const double* b, int64_t ldb) {
    const Layout& Y = c->lay;
    if (mblk < 0) return GWAS_E_INVALID;
    if (mblk > 0 && (!XR || !b || ldx < Y.n || ldb < (int64_t)Y.p * Y.t)) return GWAS_E_INVALID;
    return GWAS_OK;
}

}  // namespace

int gwas_stream_block(gwas_ctx* c, const void* XR, int64_t ldx, int64_t mblk, double* b,
                      int64_t ldb, double* var_snp, int32_t* info) {
    if (!live(c)) return GWAS_E_STATE;
    if (int rc = check_block_args(c, XR, ldx, mblk, b, ldb)) return rc;
    if (mblk == 0) return GWAS_OK;
    DeviceScope scope;
    HIPCHK(c, hipSetDevice(c->device));
    if (int rc = enqueue_block(c, XR, ldx, mblk, b, ldb, var_snp, info, c->timing)) return rc;
    HIPCHK(c, hipStreamSynchronize(c->s_h2d));
    HIPCHK(c, hipStreamSynchronize(c->s_comp));
    HIPCHK(c, hipStreamSynchronize(c->s_d2h));
    c->pending = 0;
    return collect_timing(c);
}

int gwas_stream_block_async(gwas_ctx* c, const void* XR, int64_t ldx, int64_t mblk, double* b,
                            int64_t ldb, double* var_snp, int32_t* info) {
    if (!live(c)) return GWAS_E_STATE;
    if (int rc = check_block_args(c, XR, ldx, mblk, b, ldb)) return rc;
    if (mblk == 0) return GWAS_OK;
    DeviceScope scope;
    HIPCHK(c, hipSetDevice(c->device));
    if (int rc = enqueue_block(c, XR, ldx, mblk, b, ldb, var_snp, info, c->timing)) return rc;
    c->pending += 1;
    return GWAS_OK;
}

int gwas_stream_wait(gwas_ctx* c) {
    if (!live(c)) return GWAS_E_STATE;
    DeviceScope scope;
    HIPCHK(c, hipSetDevice(c->device));
    return settle(c);
}

int gwas_stream_block_noalloc(gwas_ctx* c, const void* XR, int64_t ldx, int64_t mblk, double* b,
                              int64_t ldb, double* var_snp, int32_t* info) {
    if (!live(c)) return GWAS_E_STATE;
    if (c->lay.band > 0) return GWAS_E_INVALID;   // the banded product keeps Z in the context
    if (int rc = check_block_args(c, XR, ldx, mblk, b, ldb)) return rc;
    if (mblk == 0) return GWAS_OK;
    const Layout& Y = c->lay;
    if (Y.na_cols <= 0) {
        size_t off[6];
        noalloc_offsets(Y, TILE_N, off);
        char msg[200];
        snprintf(msg, sizeof(msg), "gwas_stream_block_noalloc: the scratch of %d SNP columns needs %zu bytes, "
                 "more than the static buffer's %zu", TILE_N, off[5], NOALLOC_SCRATCH_BYTES);
        c->err = msg;
        return GWAS_E_INVALID;
    }
    DeviceScope scope;
    HIPCHK(c, hipSetDevice(c->device));
    const size_t elem = (Y.x_dtype == GWAS_X_I8) ? 1 : 8;
    if (!(on_device(XR) && reinterpret_cast<uintptr_t>(XR) % 16 == 0 && (ldx * (int64_t)elem) % 16 == 0 &&
          ldx * (int64_t)elem <= X_DIRECT_MAX_LD_BYTES) ||
        !on_device(b) || (var_snp && !on_device(var_snp)) || (info && !on_device(info))) {
        c->err = "gwas_stream_block_noalloc: XR (16-byte aligned, ldx bytes a multiple of 16, at most 4 MiB), "
                 "b, var_snp and info must be device memory";
        return GWAS_E_INVALID;
    }
    hipStream_t s = c->s_user;
    // behind the blocks queued on the context's own streams
    HIPCHK(c, hipEventRecord(c->ev_na, c->s_comp));
    HIPCHK(c, hipStreamWaitEvent(s, c->ev_na, 0));
    size_t off[6];
    noalloc_offsets(Y, Y.na_cols, off);
    __bf16* xs = reinterpret_cast<__bf16*>(c->nscratch + off[4]);   // cut dosages (X_BF16S, X_BF16)
    // the float64 mode takes its cross terms from the partial sums (no x^T W)
    const bool red = Y.precision != GWAS_FP64;
    const SubScratch sc{reinterpret_cast<double*>(c->nscratch + off[0]), reinterpret_cast<double*>(c->nscratch + off[1]),
                        red ? reinterpret_cast<double*>(c->nscratch + off[2]) : nullptr,
                        red ? reinterpret_cast<double*>(c->nscratch + off[3]) : nullptr, Y.na_cols};
    const char* xr = static_cast<const char*>(XR);
    for (int64_t col0 = 0; col0 < mblk; col0 += Y.na_cols) {
        const int64_t cols = std::min<int64_t>(Y.na_cols, mblk - col0);
        const void* xptr = xr + (size_t)col0 * ldx * elem;
        HIPCHK(c, cut_dosages(c, xptr, ldx, cols, xs, s));
        TrmmArgs ta = trmm_args_for(c, xptr, ldx, cols, xs);
        ta.part = sc.part;
        ta.ldp = sc.ld;
        ta.sched = c->sched_na;
        ta.sched_cols = Y.na_cols;
        ta.n_sched = trmm_schedule_len(Y.n_pad, Y.na_cols, c->shape);
        HIPCHK(c, trmm_stream(ta, s));
        HIPCHK(c, finish_sub(c, sc, xptr, ldx, cols, b + (size_t)col0 * ldb, ldb,
                             var_snp ? var_snp + col0 : nullptr, info ? info + col0 : nullptr, s));
    }
    return GWAS_OK;
}

namespace {
int stream_group_impl(gwas_ctx* const* ctxs, int32_t nctx, const void* const* XR, const int64_t* ldx,
                      int64_t mblk, double* const* b, const int64_t* ldb, double* const* var_snp,
                      int32_t* const* info, int32_t flags) {
    if (!ctxs || nctx < 1 || nctx > MAX_GROUP || !XR || !ldx || !b || !ldb || mblk < 0)
        return GWAS_E_INVALID;
    if (flags & ~GWAS_GROUP_GRAPH) return GWAS_E_INVALID;
    for (int i = 0; i < nctx; ++i)
        if (!live(ctxs[i])) return GWAS_E_STATE;
    gwas_ctx* c0 = ctxs[0];
    for (int i = 0; i < nctx; ++i) {
        const gwas_ctx* c = ctxs[i];
        if (c->device != c0->device || c->at != c0->at || c->cfg != c0->cfg ||
            c->lay.x_dtype != c0->lay.x_dtype || c->lay.dev_block != c0->lay.dev_block ||
            c->lay.slices != c0->lay.slices || c->lay.band > 0)
            return GWAS_E_INVALID;
        if (!XR[i] || !b[i] || ldx[i] < c->lay.n || ldb[i] < (int64_t)c->lay.p * c->lay.t)
            return GWAS_E_INVALID;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return GWAS_E_INVALID;
    }
    if (mblk == 0) return GWAS_OK;
    DeviceScope scope;
    HIPCHK(c0, hipSetDevice(c0->device));
    for (int i = 0; i < nctx; ++i)   // blocks queued by gwas_stream_block_async
        if (int rc = settle(ctxs[i])) return rc;
    if (!c0->grp) c0->grp = new (std::nothrow) Group();
    Group* g = c0->grp;
    if (!g) return GWAS_E_OOM;
    for (int sl = 0; sl < 2; ++sl) {
        if (!g->h_args[sl]) HIPCHK(c0, hipHostMalloc((void**)&g->h_args[sl], MAX_GROUP * sizeof(TrmmArgs), 0));
        if (!g->d_args[sl]) HIPCHK(c0, hipMalloc((void**)&g->d_args[sl], MAX_GROUP * sizeof(TrmmArgs)));
    }
    std::vector<gwas_ctx*> cs(ctxs, ctxs + nctx);
    std::vector<uint64_t> key;
    // a context's generation changes with its tile shape or schedule
    // grouping (gwas_autotune): the schedule and graph are then rebuilt
    for (const gwas_ctx* c : cs) {
        key.push_back(c->id);
        key.push_back(c->gen);
    }
    hipStream_t s = c0->s_comp;
    for (int i = 0; i < nctx; ++i) HIPCHK(c0, join_user(cs[i], s));
    const int64_t blk = c0->lay.dev_block;
    const size_t elem = (c0->lay.x_dtype == GWAS_X_I8) ? 1 : 8;
    std::vector<char> direct_x(nctx), direct_out(nctx);
    for (int i = 0; i < nctx; ++i) {
        direct_x[i] = on_device(XR[i]) && (reinterpret_cast<uintptr_t>(XR[i]) % 16 == 0) &&
                      ((ldx[i] * (int64_t)elem) % 16 == 0) && ldx[i] * (int64_t)elem <= X_DIRECT_MAX_LD_BYTES;
        direct_out[i] = on_device(b[i]) && (!var_snp || !var_snp[i] || on_device(var_snp[i])) &&
                        (!info || !info[i] || on_device(info[i]));
    }
    const bool want_graph = (flags & GWAS_GROUP_GRAPH) != 0;
    const int64_t nsub = (mblk + blk - 1) / blk;
    auto ensure_schedule = [&](int64_t cols) -> int {
        if (g->key == key && g->sched_cols == cols) return GWAS_OK;
        const int64_t len = group_schedule(cs, cols, g->host_sched);
        const size_t bytes = g->host_sched.size() * sizeof(int);
        HIPCHK(c0, hipStreamSynchronize(s));   // no launch may still read the old schedule
        if (bytes > g->sched_cap) {
            HIPCHK(c0, drop(g->d_sched, hipFree));
            g->d_sched = nullptr;
            HIPCHK(c0, hipMalloc((void**)&g->d_sched, bytes));
            g->sched_cap = bytes;
        }
        HIPCHK(c0, hipMemcpy(g->d_sched, g->host_sched.data(), bytes, hipMemcpyHostToDevice));
        g->key = key;
        g->sched_cols = cols;
        g->n_sched = len;
        return GWAS_OK;
    };
    // one grouped product and every context's cross products and solves
    auto enqueue = [&](TrmmArgs* h, TrmmArgs* d, const int* sched, int64_t n_sched,
                       const std::vector<const void*>& xp, const std::vector<int64_t>& xl,
                       const std::vector<double*>& bo, const std::vector<int64_t>& lb,
                       const std::vector<double*>& vo, const std::vector<int*>& io, int64_t cols,
                       bool async_args, bool args_ready, bool x_from_args) -> int {
        if (!args_ready) {
            for (int i = 0; i < nctx; ++i) {
                h[i] = trmm_args_for(cs[i], xp[i], xl[i], cols);
                h[i].sched = sched;
                HIPCHK(c0, trmm_check(h[i], false));
            }
            if (async_args)
                HIPCHK(c0, hipMemcpyAsync(d, h, nctx * sizeof(TrmmArgs), hipMemcpyHostToDevice, s));
            else
                HIPCHK(c0, hipMemcpy(d, h, nctx * sizeof(TrmmArgs), hipMemcpyHostToDevice));
        }
        // the schedule must be the one of the contexts' current shape
        std::vector<int64_t> nrb(cs.size());
        for (size_t i = 0; i < cs.size(); ++i) nrb[i] = cs[i]->lay.n_pad / cs[0]->shape.tm;
        if (trmm_schedule_multi(nrb.data(), (int)cs.size(), cols, cs[0]->shape, nullptr) != n_sched) {
            c0->err = "grouped schedule does not match the contexts' tile shape";
            return GWAS_E_INVALID;
        }
        for (int i = 0; i < nctx; ++i)
            HIPCHK(c0, cut_dosages(cs[i], xp[i], xl[i], cols, cs[i]->xsl, s, x_from_args ? d + i : nullptr));
        TrmmArgs la = h[0];
        la.group = d;
        la.sched = sched;
        la.n_sched = n_sched;
        HIPCHK(c0, trmm_stream(la, s));
        // each context's cross products, chunk sums and solves on its own
        // stream, so the small launches of different contexts overlap; the
        // group's stream waits for all of them (in a capture these are
        // parallel branches of the graph)
        if (nctx > 1) HIPCHK(c0, hipEventRecord(c0->ev_fork, s));
        for (int i = 0; i < nctx; ++i) {
            hipStream_t si = (i == 0) ? s : cs[i]->s_comp;
            if (i > 0) HIPCHK(c0, hipStreamWaitEvent(si, c0->ev_fork, 0));
            HIPCHK(c0, finish_sub(cs[i], ctx_scratch(cs[i]), xp[i], xl[i], cols, bo[i], lb[i], vo[i], io[i], si,
                                  x_from_args ? d + i : nullptr));
            if (i > 0) {
                HIPCHK(c0, hipEventRecord(cs[i]->ev_join, si));
                HIPCHK(c0, hipStreamWaitEvent(s, cs[i]->ev_join, 0));
            }
        }
        return GWAS_OK;
    };

    for (int64_t k = 0; k < nsub; ++k) {
        const int64_t col0 = k * blk;
        const int64_t cols = std::min<int64_t>(blk, mblk - col0);
        const int slot = (int)(k & 1);
        const bool use_graph = want_graph && cols == blk;
        // in a graph the product and the cross products read the dosages
        // through the argument array: device dosages stay in place and the
        // array is updated before a replay
        int rc = ensure_schedule(cols);
        if (rc) return rc;
        std::vector<const void*> xp(nctx);
        std::vector<int64_t> xl(nctx), lb(nctx);
        std::vector<double*> bo(nctx), vo(nctx);
        std::vector<int*> io(nctx);
        const int bslot = use_graph ? 0 : slot;
        for (int i = 0; i < nctx; ++i) {
            gwas_ctx* c = cs[i];
            const char* src = static_cast<const char*>(XR[i]) + (size_t)col0 * ldx[i] * elem;
            if (direct_x[i]) {
                xp[i] = src;
                xl[i] = ldx[i];
            } else {
                HIPCHK(c0, hipMemcpy2DAsync(c->xbuf[bslot], c->lay.n_pad * elem, src, ldx[i] * elem,
                                            c->lay.n * elem, cols, hipMemcpyDefault, s));
                xp[i] = c->xbuf[bslot];
                xl[i] = c->lay.n_pad;
            }
            if (direct_out[i] && !use_graph) {
                bo[i] = b[i] + (size_t)col0 * ldb[i];
                lb[i] = ldb[i];
                vo[i] = (var_snp && var_snp[i]) ? var_snp[i] + col0 : nullptr;
                io[i] = (info && info[i]) ? info[i] + col0 : nullptr;
            } else {
                bo[i] = c->bbuf[bslot];
                lb[i] = (int64_t)c->lay.p * c->lay.t;
                vo[i] = c->vbuf[bslot];
                io[i] = c->ibuf[bslot];
            }
        }
        if (c0->timing) {
            if (int trc = timer_start(c0, s)) return trc;
        }
        if (use_graph) {
            if (!g->exec || g->graph_key != key) {
                HIPCHK(c0, hipStreamSynchronize(s));
                HIPCHK(c0, drop(g->exec, hipGraphExecDestroy));
                HIPCHK(c0, drop(g->graph, hipGraphDestroy));
                HIPCHK(c0, drop(g->d_sched_graph, hipFree));
                if (!g->h_args_graph)
                    HIPCHK(c0, hipHostMalloc((void**)&g->h_args_graph, MAX_GROUP * sizeof(TrmmArgs), 0));
                if (!g->d_args_graph) HIPCHK(c0, hipMalloc((void**)&g->d_args_graph, MAX_GROUP * sizeof(TrmmArgs)));
                // the graph's own copy of the full-width schedule and of the
                // arguments (fixed buffers), so later eager launches of other
                // widths cannot change what a replay reads
                const size_t sbytes = g->host_sched.size() * sizeof(int);
                HIPCHK(c0, hipMalloc((void**)&g->d_sched_graph, sbytes));
                HIPCHK(c0, hipMemcpy(g->d_sched_graph, g->host_sched.data(), sbytes, hipMemcpyHostToDevice));
                // arguments are uploaded synchronously before capture begins
                for (int i = 0; i < nctx; ++i) {
                    g->h_args_graph[i] = trmm_args_for(cs[i], xp[i], xl[i], cols);
                    g->h_args_graph[i].sched = g->d_sched_graph;
                    HIPCHK(c0, trmm_check(g->h_args_graph[i], false));
                }
                HIPCHK(c0, hipMemcpy(g->d_args_graph, g->h_args_graph, nctx * sizeof(TrmmArgs),
                                     hipMemcpyHostToDevice));
                // (checked directly: a capture must never be left open)
                if (const hipError_t eb = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal))
                    return fail_hip(c0, eb, "hipStreamBeginCapture");
                const int erc = enqueue(g->h_args_graph, g->d_args_graph, g->d_sched_graph, g->n_sched, xp, xl,
                                        bo, lb, vo, io, cols, false, true, true);
                hipGraph_t graph = nullptr;
                const hipError_t ec = hipStreamEndCapture(s, &graph);
                g->graph = graph;   // owned by the group from here on, whatever fails below
                if (erc) return erc;
                HIPCHK(c0, ec);
                HIPCHK(c0, hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
                g->graph_key = key;
                g->graph_x = xp;
                g->graph_ldx = xl;
            } else if (g->graph_x != xp || g->graph_ldx != xl) {
                // new dosage pointers: upload the argument array, in stream
                // order behind the replays that read the old one, from a
                // pinned copy that no queued upload still reads
                if (!g->h_args_upd[slot])
                    HIPCHK(c0, hipHostMalloc((void**)&g->h_args_upd[slot], MAX_GROUP * sizeof(TrmmArgs), 0));
                if (k >= 2) HIPCHK(c0, hipEventSynchronize(c0->ev_done[slot]));
                for (int i = 0; i < nctx; ++i) {
                    TrmmArgs a = g->h_args_graph[i];
                    a.Xd = xp[i];
                    a.ldxd = xl[i];
                    if (!x_cut(a.xt)) {   // cut dosages stay in the context's buffer
                        a.X = xp[i];
                        a.ldx = xl[i];
                    }
                    HIPCHK(c0, trmm_check(a, false));
                    g->h_args_upd[slot][i] = a;
                }
                HIPCHK(c0, hipMemcpyAsync(g->d_args_graph, g->h_args_upd[slot], nctx * sizeof(TrmmArgs),
                                          hipMemcpyHostToDevice, s));
                g->graph_x = xp;
                g->graph_ldx = xl;
            }
            HIPCHK(c0, hipGraphLaunch(g->exec, s));
        } else {
            if (k >= 2) HIPCHK(c0, hipEventSynchronize(c0->ev_done[slot]));   // slot's arguments free
            const int erc = enqueue(g->h_args[slot], g->d_args[slot], g->d_sched, g->n_sched, xp, xl, bo, lb,
                                    vo, io, cols, true, false, false);
            if (erc) return erc;
        }
        if (c0->timing) {
            if (int trc = timer_stop(c0, s, cols * nctx)) return trc;
        }
        for (int i = 0; i < nctx; ++i) {
            if (direct_out[i] && !use_graph) continue;
            const int64_t pt = (int64_t)cs[i]->lay.p * cs[i]->lay.t;
            HIPCHK(c0, hipMemcpy2DAsync(b[i] + (size_t)col0 * ldb[i], ldb[i] * 8, bo[i], pt * 8, pt * 8, cols,
                                        hipMemcpyDefault, s));
            if (var_snp && var_snp[i])
                HIPCHK(c0, hipMemcpyAsync(var_snp[i] + col0, vo[i], cols * 8, hipMemcpyDefault, s));
            if (info && info[i])
                HIPCHK(c0, hipMemcpyAsync(info[i] + col0, io[i], cols * 4, hipMemcpyDefault, s));
        }
        HIPCHK(c0, hipEventRecord(c0->ev_done[slot], s));
    }
    HIPCHK(c0, hipStreamSynchronize(s));
    return collect_timing(c0);
}
}  // namespace

int gwas_stream_group(gwas_ctx* const* ctxs, int32_t nctx, const void* const* XR, const int64_t* ldx,
                      int64_t mblk, double* const* b, const int64_t* ldb, double* const* var_snp,
                      int32_t* const* info, int32_t flags) {
    const int rc = stream_group_impl(ctxs, nctx, XR, ldx, mblk, b, ldb, var_snp, info, flags);
    // a device error poisons the first context; the others' queued copies
    // are waited for too
    if (rc == GWAS_E_HIP || rc == GWAS_E_OOM)
        for (int i = 1; i < nctx; ++i)
            if (ctxs[i] && ctxs[i]->magic == CTX_MAGIC) drain(ctxs[i]);
    return rc;
}

int gwas_autotune(gwas_ctx* c, const void* XR, int64_t ldx, int64_t cols, int32_t* best_cfg,
                  int32_t* best_rgroup) {
    if (!live(c)) return GWAS_E_STATE;
    if (c->lay.band > 0) return GWAS_E_INVALID;   // one tile shape
    const Layout& Y = c->lay;
    if (!XR || ldx < Y.n || cols < 1) return GWAS_E_INVALID;
    cols = std::min<int64_t>(cols, Y.dev_block);
    DeviceScope scope;
    HIPCHK(c, hipSetDevice(c->device));
    if (int rc = settle(c)) return rc;   // blocks queued by gwas_stream_block_async
    HIPCHK(c, join_user(c, c->s_comp));
    HIPCHK(c, hipStreamSynchronize(c->s_comp));
    const int xt = prod_xt_of(Y.precision, Y.x_dtype);   // the product's dosage operand
    const char* cache = getenv("GWAS_TUNE_CACHE");
    char keyline[160];
    snprintf(keyline, sizeof(keyline), "gfx950 n_pad=%lld precision=%d x_dtype=%d cols=%lld",
             (long long)Y.n_pad, Y.precision, Y.x_dtype, (long long)cols);
    int best = -1, best_rg = 0;
    int64_t best_sub = 0;
    if (cache) {
        if (FILE* f = fopen(cache, "r")) {
            char line[256];
            while (fgets(line, sizeof(line), f)) {
                const size_t kl = strlen(keyline);
                int v = -1, r = 0;
                long long w = Y.dev_block;   // lines without a width keep dev_block
                if (strncmp(line, keyline, kl) == 0 &&
                    sscanf(line + kl, " cfg=%d rgroup=%d sub=%lld", &v, &r, &w) >= 2 &&
                    trmm_cfg_valid(c->at, xt, v) && r >= 1 && r <= 32 && w >= TILE_N && w <= Y.dev_block &&
                    w % TILE_N == 0) {
                    best = v;
                    best_rg = r;
                    best_sub = w;
                }
            }
            fclose(f);
        }
    }
    if (best_rg == 0) {
        const size_t elem = (Y.x_dtype == GWAS_X_I8) ? 1 : 8;
        const void* xptr = XR;
        int64_t xld = ldx;
        if (!(on_device(XR) && reinterpret_cast<uintptr_t>(XR) % 16 == 0 && (ldx * (int64_t)elem) % 16 == 0 &&
              ldx * (int64_t)elem <= X_DIRECT_MAX_LD_BYTES)) {
            HIPCHK(c, hipMemcpy2D(c->xbuf[0], Y.n_pad * elem, XR, ldx * elem, Y.n * elem, cols, hipMemcpyDefault));
            xptr = c->xbuf[0];
            xld = Y.n_pad;
        }
        // float64 dosages of the bfloat16 products: the cut dosages the products read
        HIPCHK(c, cut_dosages(c, xptr, xld, cols, c->xsl, c->s_comp));
        hipEvent_t e0, e1;
        HIPCHK(c, hipEventCreate(&e0));
        HIPCHK(c, hipEventCreate(&e1));
        float best_ms = 0.f;
        // every admissible tile shape with every candidate row group of the
        // schedule
        for (int cfg = 0; cfg < trmm_cfg_limit(); ++cfg) {
            if (!trmm_cfg_valid(c->at, xt, cfg)) continue;
            for (int rg : RGROUP_CANDIDATES) {
                c->gen += 1;
                c->cfg = cfg;
                c->rgroup = rg;
                c->shape = trmm_geom(c->at, xt, c->cfg, Y.slices, rg);
                int rc = upload_schedule(c, cols, c->sched_tail, c->host_tail);
                if (rc) return rc;
                TrmmArgs ta = trmm_args_for(c, xptr, xld, cols);
                ta.sched = c->sched_tail;
                HIPCHK(c, trmm_stream(ta, c->s_comp));                  // warm-up
                HIPCHK(c, hipEventRecord(e0, c->s_comp));
                HIPCHK(c, trmm_stream(ta, c->s_comp));
                HIPCHK(c, hipEventRecord(e1, c->s_comp));
                HIPCHK(c, hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
                if (best_rg == 0 || ms < best_ms) {
                    best = cfg;
                    best_rg = rg;
                    best_ms = ms;
                }
            }
        }
        // the sub-block width with that shape: dev_block, a half or a
        // quarter of it (whole multiples of 128 columns that fit the timing
        // block), by the product's time per column over whole sub-blocks
        c->gen += 1;
        c->cfg = best;
        c->rgroup = best_rg;
        c->shape = trmm_geom(c->at, xt, c->cfg, Y.slices, best_rg);
        double best_per_col = 0.0;
        for (int d : {1, 2, 4}) {
            const int64_t w = Y.dev_block / d / TILE_N * TILE_N;
            if (w < TILE_N || w > cols) continue;
            const int64_t reps = cols / w;
            int rc = upload_schedule(c, w, c->sched_tail, c->host_tail);
            if (rc) return rc;
            auto launch_all = [&]() -> int {
                for (int64_t q = 0; q < reps; ++q) {
                    TrmmArgs ta = trmm_args_for(c, static_cast<const char*>(xptr) + (size_t)(q * w) * xld * elem,
                                                xld, w, c->xsl ? c->xsl + (size_t)(q * w) * x_cut_ld(xt, Y.n_pad) : nullptr);
                    ta.sched = c->sched_tail;
                    HIPCHK(c, trmm_stream(ta, c->s_comp));
                }
                return GWAS_OK;
            };
            if (int lrc = launch_all()) return lrc;                 // warm-up
            HIPCHK(c, hipEventRecord(e0, c->s_comp));
            if (int lrc = launch_all()) return lrc;
            HIPCHK(c, hipEventRecord(e1, c->s_comp));
            HIPCHK(c, hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
            const double per_col = ms / (double)(reps * w);
            if (best_sub == 0 || per_col < best_per_col) {
                best_sub = w;
                best_per_col = per_col;
            }
        }
        if (best_sub == 0) best_sub = Y.dev_block;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (cache) {
            if (FILE* f = fopen(cache, "a")) {
                fprintf(f, "%s cfg=%d rgroup=%d sub=%lld ms=%.3f\n", keyline, best, best_rg, (long long)best_sub,
                        best_ms);
                fclose(f);
            }
        }
    }
    c->gen += 1;
    c->cfg = best < 0 ? 0 : best;
    c->rgroup = best_rg;
    c->shape = trmm_geom(c->at, xt, c->cfg, Y.slices, best_rg);
    c->tail_cols = -1;
    c->sub = best_sub > 0 ? best_sub : Y.dev_block;
    int rc = upload_schedule(c, c->sub, c->sched, c->host_sched);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->s_comp));
    rc = upload_noalloc_schedule(c);
    if (rc) return rc;
    if (best_rgroup) *best_rgroup = best_rg;
    if (best_cfg) *best_cfg = best;
    return GWAS_OK;
}

int gwas_backward_begin(gwas_ctx* c) {
    if (!live(c)) return GWAS_E_STATE;
    if (c->lay.band > 0) return GWAS_E_INVALID;   // needs the dense inverse factor
    const Layout& Y = c->lay;
    if (Y.t != 1) return GWAS_E_INVALID;
    DeviceScope scope;
    HIPCHK(c, hipSetDevice(c->device));
    if (int rc = settle(c)) return rc;   // blocks queued by gwas_stream_block_async
    hipStream_t s = c->s_comp;
    if (!c->back) {
        c->back = new (std::nothrow) Back();
        if (!c->back) return GWAS_E_OOM;
    }
    Back* B = c->back;
    const int p = Y.p;
    const int64_t np = Y.n_pad, blk = Y.dev_block;
    const int xt = (Y.x_dtype == GWAS_X_I8) ? X_I8 : X_F64;
    const TrmmShape sh = trmm_geom(A_F64, xt, trmm_default_cfg(A_F64, xt), 0);
    if (!B->mem) {
        B->npb = np / sh.part_rows;
        size_t o = 0;
        std::vector<std::pair<double**, size_t>> parts = {
            {&B->Minv, (size_t)np * np}, {&B->W, (size_t)np * p}, {&B->GW, (size_t)(p - 1) * p},
            {&B->part, (size_t)B->npb * (p + 1) * blk}, {&B->red, (size_t)chunks_of(B->npb) * (p + 1) * blk},
            {&B->xw, (size_t)p * blk},
            {&B->contrib, (size_t)(p + 1) * blk}, {&B->coef, (size_t)blk}, {&B->g, (size_t)np},
            {&B->acc, (size_t)(p + 1)}, {&B->v, (size_t)np}, {&B->gy, (size_t)np},
            {&B->sb, (size_t)p * blk}, {&B->sv, (size_t)blk}, {&B->sgb, (size_t)p * blk},
            {&B->sgv, (size_t)blk}};
        std::vector<size_t> offs;
        for (auto& pr : parts) {
            offs.push_back(o);
            o = align_up(o + pr.second * 8, 256);
        }
        const size_t off_si = o;
        o = align_up(o + (size_t)blk * 4, 256);
        if (hipMalloc(&B->mem, o) != hipSuccess) {
            (void)hipGetLastError();
            B->mem = nullptr;
            c->err = "reverse-pass workspace allocation failed";
            return GWAS_E_OOM;
        }
        for (size_t i = 0; i < parts.size(); ++i) *parts[i].first = (double*)(B->mem + offs[i]);
        B->si = (int*)(B->mem + off_si);
        B->ready = false;
    }
    HIPCHK(c, join_user(c, s));
    if (!B->ready) {
        // M^-1 = U U^T (U = L^-T upper): K range [max(m0, n0), n_pad)
        GemmArgs g{np, np, np, c->U, Y.ld, 'N', c->U, Y.ld, 'T', B->Minv, np, 1.0, 0.0,
                   KR_A_UPPER | KR_B_LOWER, 0};
        HIPCHK(c, gemm_f64(g, s));
        // W = U C with C = L^-1 [X_L | y]
        g = GemmArgs{np, p, np, c->U, Y.ld, 'N', c->C, np, 'N', B->W, np, 1.0, 0.0, KR_A_UPPER, 0};
        HIPCHK(c, gemm_f64(g, s));
        // [W_L^T W_L | W_L^T w_y]
        g = GemmArgs{p - 1, p, np, B->W, np, 'T', B->W, np, 'N', B->GW, p - 1, 1.0, 0.0, 0, 0};
        HIPCHK(c, gemm_f64(g, s));
        B->ready = true;
    }
    HIPCHK(c, hipMemsetAsync(B->g, 0, (size_t)np * 8, s));
    HIPCHK(c, hipMemsetAsync(B->acc, 0, (size_t)(p + 1) * 8, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return GWAS_OK;
}

int gwas_backward_block(gwas_ctx* c, const void* XR, int64_t ldx, int64_t mblk, const double* b,
                        int64_t ldb, const double* var_snp, const int32_t* info, const double* gb,
                        int64_t ldgb, const double* gvar) {
    if (!live(c)) return GWAS_E_STATE;
    if (!c->back || !c->back->ready) return GWAS_E_STATE;
    const Layout& Y = c->lay;
    const int p = Y.p;
    if (mblk < 0 || (mblk > 0 && (!XR || !b || !var_snp || !info || !gb)) || ldx < Y.n || ldb < p ||
        ldgb < p)
        return GWAS_E_INVALID;
    if (mblk == 0) return GWAS_OK;
    DeviceScope scope;
    HIPCHK(c, hipSetDevice(c->device));
    if (int rc = settle(c)) return rc;   // blocks queued by gwas_stream_block_async
    Back* B = c->back;
    hipStream_t s = c->s_comp;
    HIPCHK(c, join_user(c, s));
    const size_t elem = (Y.x_dtype == GWAS_X_I8) ? 1 : 8;
    const int xt = (Y.x_dtype == GWAS_X_I8) ? X_I8 : X_F64;
    const int cfg = trmm_default_cfg(A_F64, xt);
    const TrmmShape sh = trmm_geom(A_F64, xt, cfg, 0);
    const bool direct_x = on_device(XR) && (reinterpret_cast<uintptr_t>(XR) % 16 == 0) &&
                          ((ldx * (int64_t)elem) % 16 == 0) && ldx * (int64_t)elem <= X_DIRECT_MAX_LD_BYTES;
    const int64_t blk = Y.dev_block;
    for (int64_t col0 = 0; col0 < mblk; col0 += blk) {
        const int64_t cols = std::min<int64_t>(blk, mblk - col0);
        const char* src = static_cast<const char*>(XR) + (size_t)col0 * ldx * elem;
        const void* xptr = src;
        int64_t xld = ldx;
        if (!direct_x) {
            HIPCHK(c, hipMemcpy2DAsync(c->xbuf[0], Y.n_pad * elem, src, ldx * elem, Y.n * elem, cols,
                                       hipMemcpyDefault, s));
            xptr = c->xbuf[0];
            xld = Y.n_pad;
        }
        // forward results and cotangents of this sub-block into device scratch
        HIPCHK(c, hipMemcpy2DAsync(B->sb, p * 8, b + (size_t)col0 * ldb, ldb * 8, p * 8, cols, hipMemcpyDefault, s));
        HIPCHK(c, hipMemcpy2DAsync(B->sgb, p * 8, gb + (size_t)col0 * ldgb, ldgb * 8, p * 8, cols,
                                   hipMemcpyDefault, s));
        HIPCHK(c, hipMemcpyAsync(B->sv, var_snp + col0, cols * 8, hipMemcpyDefault, s));
        HIPCHK(c, hipMemcpyAsync(B->si, info + col0, cols * 4, hipMemcpyDefault, s));
        if (gvar) HIPCHK(c, hipMemcpyAsync(B->sgv, gvar + col0, cols * 8, hipMemcpyDefault, s));
        // w = M^-1 x with the sums w^T [W_L | w_y] and w^T w
        std::vector<int> sched((size_t)(2 * trmm_schedule_len(Y.n_pad, cols, sh)));
        const int64_t ns = trmm_schedule(Y.n_pad, cols, sh, sched.data(), (int64_t)sched.size() / 2);
        if (ns < 0 || (size_t)(2 * ns) * sizeof(int) > Y.sched_len * 2 * sizeof(int)) {
            c->err = "reverse-pass schedule does not fit";
            return GWAS_E_INVALID;
        }
        HIPCHK(c, hipMemcpy(c->sched_tail, sched.data(), sched.size() * sizeof(int), hipMemcpyHostToDevice));
        c->tail_cols = -1;
        TrmmArgs ta{};
        ta.at = A_F64;
        ta.xt = xt;
        ta.cfg = cfg;
        ta.Ut = B->Minv;
        ta.ldu = Y.n_pad;
        ta.n_pad = Y.n_pad;
        ta.X = xptr;
        ta.ldx = xld;
        ta.n = Y.n;
        ta.cols = cols;
        ta.C = B->W;
        ta.ldc = Y.n_pad;
        ta.Qc = p;
        ta.with_cross = 1;
        ta.part = B->part;
        ta.ldp = blk;
        ta.sched = c->sched_tail;
        ta.n_sched = ns;
        ta.full_k = 1;
        HIPCHK(c, trmm_stream(ta, s));
        HIPCHK(c, snp_cross_w(xt, xptr, xld, Y.n, cols, B->W, Y.n_pad, p, B->xw, blk, nullptr, 0, s));
        HIPCHK(c, partial_chunks(B->part, blk, Y.n_pad / sh.part_rows, p + 1, cols, PART_CHUNK, B->red, blk, s));
        BackArgs ba{};
        ba.p = p;
        ba.cols = cols;
        ba.part = B->red;   // chunk totals of the partial sums
        ba.ldp = blk;
        ba.npb = chunks_of(Y.n_pad / sh.part_rows);
        ba.xw = B->xw;
        ba.ldxw = blk;
        ba.consts = c->consts;
        ba.G = B->GW;
        ba.gy0 = B->GW + (size_t)(p - 1) * (p - 1);
        ba.b = B->sb;
        ba.ldb = p;
        ba.var = B->sv;
        ba.info = B->si;
        ba.gb = B->sgb;
        ba.ldgb = p;
        ba.gv = gvar ? B->sgv : nullptr;
        ba.contrib = B->contrib;
        ba.ldc = blk;
        ba.coef = B->coef;
        HIPCHK(c, snp_backward(ba, s));
        HIPCHK(c, sum_columns(B->contrib, blk, p + 1, cols, B->acc, s));
        HIPCHK(c, dosage_gemv(xt, xptr, xld, Y.n, cols, B->coef, B->g, s));
        HIPCHK(c, hipStreamSynchronize(s));   // scratch and schedule are reused by the next sub-block
    }
    return GWAS_OK;
}

int gwas_backward_end(gwas_ctx* c, double* gy, double* tr_mbar, double* ip_mbar_m) {
    if (!live(c)) return GWAS_E_STATE;
    if (!c->back || !c->back->ready) return GWAS_E_STATE;
    const Layout& Y = c->lay;
    Back* B = c->back;
    hipStream_t s = c->s_comp;
    DeviceScope scope;
    HIPCHK(c, hipSetDevice(c->device));
    if (int rc = settle(c)) return rc;   // blocks queued by gwas_stream_block_async
    HIPCHK(c, join_user(c, s));
    const int p = Y.p;
    const int64_t np = Y.n_pad;
    // v = X_L a_L + X_R a_SNP, then dl/dy = M^-1 v
    HIPCHK(c, hipMemcpyAsync(B->v, B->g, (size_t)np * 8, hipMemcpyDeviceToDevice, s));
    GemmArgs g{np, 1, p - 1, c->XY, np, 'N', B->acc, p - 1, 'N', B->v, np, 1.0, 1.0, 0, 0};
    HIPCHK(c, gemm_f64(g, s));
    g = GemmArgs{np, 1, np, B->Minv, np, 'N', B->v, np, 'N', B->gy, np, 1.0, 0.0, 0, 0};
    HIPCHK(c, gemm_f64(g, s));
    double acc2[2] = {0.0, 0.0};
    HIPCHK(c, hipMemcpyAsync(acc2, B->acc + (p - 1), 16, hipMemcpyDeviceToHost, s));
    if (gy) HIPCHK(c, hipMemcpyAsync(gy, B->gy, (size_t)Y.n * 8, hipMemcpyDefault, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (tr_mbar) *tr_mbar = acc2[0];
    if (ip_mbar_m) *ip_mbar_m = acc2[1];
    return GWAS_OK;
}

int gwas_test_inject_fault(gwas_ctx* c, int64_t k) {
    if (!live(c)) return GWAS_E_STATE;
    if (k < 0) return GWAS_E_INVALID;
    c->inject_at = k;
    c->injected = false;
    return GWAS_OK;
}

int gwas_free(gwas_ctx* c) {
    if (!c) return GWAS_OK;
    if (c->magic != CTX_MAGIC) return GWAS_E_STATE;
    DeviceScope scope;
    (void)hipSetDevice(c->device);
    release(c);
    c->magic = CTX_DEAD;
    delete c;
    return GWAS_OK;
}

const char* gwas_strerror(int code) {
    switch (code) {
        case GWAS_OK: return "ok";
        case GWAS_E_INVALID: return "invalid argument";
        case GWAS_E_NOT_SPD: return "M is not positive definite";
        case GWAS_E_RANK_XL: return "X_L^T M^-1 X_L is not positive definite (X_L rank deficient)";
        case GWAS_E_NO_DEVICE: return "no usable gfx950 device";
        case GWAS_E_HIP: return "HIP runtime error";
        case GWAS_E_OOM: return "device memory exhausted";
        case GWAS_E_STATE: return "context is NULL, freed or poisoned";
        case GWAS_E_WORKSPACE: return "workspace smaller than gwas_workspace_bytes";
        default: return "unknown status";
    }
}

int64_t gwas_info(const gwas_ctx* c) {
    if (!c || c->magic != CTX_MAGIC) return -1;
    return c->info;
}

const char* gwas_last_error(const gwas_ctx* c) {
    if (!c || c->magic != CTX_MAGIC) return "invalid context";
    return c->err.c_str();
}

int gwas_set_timing(gwas_ctx* c, int32_t enable) {
    if (!live(c)) return GWAS_E_STATE;
    {
        DeviceScope scope;
        HIPCHK(c, hipSetDevice(c->device));
        if (int rc = settle(c)) return rc;   // queued blocks are timed under the old setting
    }
    c->timing = enable != 0;
    c->t_launches = 0;
    c->t_cols = 0;
    c->t_ms = 0.0;
    return GWAS_OK;
}

int gwas_kernel_time(gwas_ctx* c, int64_t* launches, double* total_ms, int64_t* columns) {
    if (!live(c)) return GWAS_E_STATE;
    if (launches) *launches = c->t_launches;
    if (total_ms) *total_ms = c->t_ms;
    if (columns) *columns = c->t_cols;
    return GWAS_OK;
}

int gwas_query(const gwas_ctx* c, int64_t* n_pad, int64_t* dev_block, int32_t* device) {
    if (!c || c->magic != CTX_MAGIC) return GWAS_E_STATE;
    if (n_pad) *n_pad = c->lay.n_pad;
    if (dev_block) *dev_block = c->sub > 0 ? c->sub : c->lay.dev_block;
    if (device) *device = c->device;
    return GWAS_OK;
}

}  // extern "C"
