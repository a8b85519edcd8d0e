// Host runtime of the rAPDB library: handles, device memory, the device-resident solve loop,
// evaluations, and continuous batching.  Implements include/qcqp.h.
//
// Paper: "Restarted Accelerated Primal-Dual Algorithms with Adaptive Stepsizes for Nonlinear
// Conic Constrained Convex Optimization" (arXiv 2605.29291); the method is Algorithm 2
// (rAPDB) around the APDB-yx routine of §3.2 or the APDB-xy routine of Algorithm 1; see
// kernels.hip for the per-kernel mapping.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/qcqp.h"
#include "qcqp_device.h"

using namespace qcqp;

namespace {

thread_local std::string g_err;

qcqp_status fail(qcqp_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(e_ == hipErrorOutOfMemory ? QCQP_E_NOMEM : QCQP_E_DEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                   \
    } while (0)

int elem_size(int dt) { return dt == DT_F64 ? 8 : (dt == DT_F32 ? 4 : 2); }
int vec_width(int dt) { return 16 / elem_size(dt); }
int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

bool prepared = false;
int prepared_dev = -1;
int max_lds = 64 * 1024;   // dynamic LDS a workgroup may request on this device
int num_cus = 0;           // compute units of the device

qcqp_status ensure_prepared()
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (!prepared || prepared_dev != dev) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess || v <= 0)
            HIPCHK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        max_lds = v;
        HIPCHK(hipDeviceGetAttribute(&num_cus, hipDeviceAttributeMultiprocessorCount, dev));
        HIPCHK(prepare_kernels(v));
        HIPCHK(prepare_fista_coop(v));
        prepared = true;
        prepared_dev = dev;
    }
    return QCQP_OK;
}

// order the library's work stream after everything already queued on the caller's stream
hipError_t join_streams(hipStream_t work, hipStream_t user, hipEvent_t ev)
{
    hipError_t e = hipEventRecord(ev, user);
    if (e == hipSuccess) e = hipStreamWaitEvent(work, ev, 0);
    return e;
}

// capture the launches `fn` enqueues on `s` into an instantiated graph
template <typename F>
hipError_t capture_graph(hipStream_t s, F fn, hipGraphExec_t *out)
{
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t el = fn(s);
    e = hipStreamEndCapture(s, &g);
    if (el != hipSuccess) e = el;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr double CACHE_RESIDENT_BYTES = 256e6;   // Infinity Cache (MALL) of one MI355X
// largest accepted asymmetry of a stored matrix, relative to its largest entry
constexpr double SYMMETRY_TOL = 1e-12;

// Lanes per row and rows per tile for a stack of `rows` rows of n elements of type dt.
// A lane should issue at least one full batch of 8 loads per row, so short rows share a wave
// (32 or 16 lanes per row).  Tiles hold ~128 KB of the stack, rounded to whole block steps
// (every lane group streams its R rows), and there are at least ~1024 of them when the stack
// allows it, so that the pass grid splits into nearly equal contiguous ranges.
void tile_shape(int64_t n, int dt, int64_t rows, int *lpr, int *rows_per_tile)
{
    const int64_t vpr = (n + vec_width(dt) - 1) / vec_width(dt);   // 16-byte vectors per row
    // lanes per row: the widest group (64 .. 8 lanes) in which each lane still streams `loads`
    // vectors of a row
    constexpr int loads = 8, min_lpr = 8;
    int l = min_lpr;
    for (int c = 64; c > min_lpr; c /= 2)
        if (vpr >= (int64_t)loads * c) {
            l = c;
            break;
        }
    const int step = (PASS_BS / l) * pass_rows_per_step(dt);   // rows one block covers at once
    const int64_t row_bytes = n * elem_size(dt);
    int64_t r = std::max<int64_t>(1, (128 * 1024) / std::max<int64_t>(row_bytes, 1));
    r = std::min<int64_t>(r, std::max<int64_t>(1, rows / 1024));
    r = round_up(std::max<int64_t>(r, step), step);
    *lpr = l;
    *rows_per_tile = (int)r;
}

// Pass grid.  One round is the resident block count (CUs x pass blocks per CU).  With one
// byte-balanced range per resident block, blocks on slower CUs finished up to twice as late as
// the fastest (config 2: 250 to 500 us), so when at least two blocks fit on a CU the grid takes
// up to four rounds and the hardware hands the later ranges to whichever CUs free up first.
// Every block stages w ((B + 1) n FP64 values from L2) when it starts: a round is added only
// while each block still streams at least ten times those bytes.  With one block per CU a new
// block's staging would leave its CU idle, so the grid stays at one round.
constexpr int PASS_GRID_ROUNDS = 4;

int pass_grid_for(int B, int dtype, int max_nw, double stack_bytes)
{
    const int occ = pass_blocks_per_cu(B, dtype, max_nw);
    const int base = std::max(1, num_cus) * occ;
    if (occ < 2) return base;
    const double stage = (double)(B + 1) * max_nw * 8.0;
    for (int k = PASS_GRID_ROUNDS; k > 1; k /= 2)
        if (stack_bytes / ((double)base * k) >= 10.0 * stage) return base * k;
    return base;
}

// First tile of each of the `grid` pass blocks so that every block streams nearly the same
// number of bytes: block b starts at the first tile whose preceding bytes reach b/grid of the
// total.  Tiles of different requests carry different bytes (row lengths, storage), so equal
// tile counts would leave blocks unequal.
std::vector<int> balanced_starts(const std::vector<int64_t> &tile_bytes, int grid)
{
    const int nt = (int)tile_bytes.size();
    std::vector<int> st(grid + 1, nt);
    double total = 0.0;
    for (int64_t b : tile_bytes) total += (double)b;
    double acc = 0.0;
    int t = 0;
    for (int b = 0; b < grid; ++b) {
        const double target = total * (double)b / (double)grid;
        while (t < nt && acc + 0.5 * (double)tile_bytes[t] < target) acc += (double)tile_bytes[t++];
        st[b] = t;
    }
    st[grid] = nt;
    return st;
}

}  // namespace

// Doubles of G_xi scratch for dimension n: H (n x ldh, ldh = n rounded up to 16), six vectors
// of n rounded up to 32, two partial sums per block of the inner loop and 64 control words
// (the inner loop's grid barrier lives in the last of them).
constexpr int64_t gap_scratch_doubles(int64_t n)
{
    return n * ((n + 15) / 16 * 16) + 6 * ((n + 31) / 32 * 32) + 2 * GAP_MAX_BLOCKS + 64;
}

// ---------------------------------------------------------------------------------------
// Static scratch of qcqp_eval_gap_noalloc: G_xi scratch for n <= QCQP_NOALLOC_MAX_N, one copy
// per GPU for the life of the process.  In host code `scratch` names a host-side stand-in, so
// its device address is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that address is handed to kernels and copies.

static __device__ __align__(256) double scratch[gap_scratch_doubles(QCQP_NOALLOC_MAX_N)];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_addr[SCRATCH_MAX_DEVICES] = {};

qcqp_status static_scratch_for(int dev, double **out)
{
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(QCQP_E_DEVICE, "device id %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        int cur = 0;
        HIPCHK(hipGetDevice(&cur));
        if (cur != dev) HIPCHK(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) HIPCHK(hipSetDevice(cur));
        if (e != hipSuccess || !p)
            return fail(QCQP_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_addr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_addr[dev];
    return QCQP_OK;
}
}  // namespace

// ---------------------------------------------------------------------------------------

struct qcqp_handle {
    int dev = 0;
    hipStream_t stream = nullptr;     // the library's own work stream (default priority)
    hipStream_t ustream = nullptr;    // the caller's stream (options.stream)
    hipEvent_t ev_join = nullptr;
    hipGraphExec_t gexec = nullptr;   // captured chunk of trial groups (solve)
    int64_t gexec_groups = 0;
    qcqp_options opt{};
    int64_t n = 0, m = 0, p = 0, ny = 0, nq = 0, ld = 0, nw = 0;
    int has_q0 = 1, on_device = 0, dtype = DT_F64, incremental = 0, B = 1;
    void *dQ = nullptr;
    char *arena = nullptr;
    size_t arena_bytes = 0, q_bytes = 0;
    Slot hslot{};             // canonical buffer assignment; uploaded at the start of a run
    Slot *dslot = nullptr;    // device copy used by single solves
    Slot *dslot_eval = nullptr;   // device slot of point evaluations (never the running one)
    int *dlive0 = nullptr;        // device live list {0}: the single slot of a standalone run
    Tile *dtiles = nullptr;
    int *dstarts = nullptr;   // balanced first tile per pass block (pass grid + 1 entries)
    std::vector<Tile> tiles;  // slot field 0
    int nblk_step = 1;
    int pass_grid = 1, nt = 0;
    double *d_ueval = nullptr, *d_geval = nullptr, *d_grad = nullptr, *d_kpart = nullptr,
           *d_out6 = nullptr, *d_xe = nullptr, *d_ye = nullptr;
    Slot *h_poll = nullptr;   // pinned: two status snapshots (pipelined polls)
    hipEvent_t ev_snap[2] = {nullptr, nullptr};   // recorded after each snapshot copy
    double *h_out = nullptr;  // pinned scratch (16 doubles)
    qcqp_batch *owner = nullptr;
    double *gap_mem = nullptr;  // G_xi scratch: H (n x ldh), 6 vectors, partials, control
    size_t gap_bytes = 0;
    double *gap_ctl = nullptr;  // control words of the last G_xi enqueued (in gap_mem)
    // options.sym_pass: the packed upper-triangle copy of the stack, its per-tile results and
    // the output row base of each stored matrix
    bool use_sym = false;
    SymPass sym{};
    double *dP = nullptr, *dws = nullptr;
    int32_t *dubase = nullptr;
    size_t sym_bytes = 0;
    // 16-bit storage: the device copy of `sym` and the launch description of a single solve
    SymPass *dsym = nullptr;
    Sym16Launch s16{};
    // the packed pass to launch, by storage type
    const SymPass *sym64() const { return use_sym && dtype == DT_F64 ? &sym : nullptr; }
    const Sym16Launch *sym16() const { return use_sym && dtype != DT_F64 ? &s16 : nullptr; }
};

struct qcqp_batch {
    qcqp_options opt{};
    size_t budget = 0;
    int64_t max_slots = 0;
    int dev = 0;
    hipStream_t stream = nullptr;     // own work stream
    hipStream_t ustream = nullptr;    // caller's stream
    hipEvent_t ev_join = nullptr;
    hipGraphExec_t gexec = nullptr;   // captured chunk of trial groups for the current live set
    int64_t gexec_groups = 0;
    std::vector<qcqp_handle *> handles;   // per slot, nullptr = free
    std::vector<int> finished;            // per slot: status already reported finished
    Slot *dslots = nullptr;
    Slot *h_poll = nullptr;               // pinned copy of all slots
    Tile *dtiles = nullptr;
    size_t tiles_cap = 0;
    int *dstarts = nullptr;               // balanced first tile per pass block
    size_t starts_cap = 0;
    std::vector<int> starts_host;         // kept alive until the copy above has run
    int *dlive = nullptr;                 // device list of live slot ids (max_slots entries)
    int nlive = 0;
    int ntiles = 0, max_nblk = 1, max_ny = 1, max_nw = 2, max_epi = 1;
    int variants = HAS_YX;                // HAS_YX | HAS_XY over the live slots
    int pass_grid = 1, nt = 0;
    bool dirty = true;
    // pass timing (options.timing): kernel seconds and algorithmic bytes streamed
    std::vector<hipEvent_t> ev;
    double pass_seconds = 0.0, pass_bytes = 0.0;
    int64_t passes = 0;
    std::vector<int64_t> last_passes;     // per slot, device pass counter at the last poll
    hipStream_t gstream = nullptr;        // G_xi evaluations of pending slots (default priority)
    std::vector<int> gap_busy;            // per slot: a G_xi is in flight on gstream
    std::vector<hipEvent_t> gev;          // per slot: recorded after that G_xi
    // slots whose handles run the 16-bit packed pass (sym_pass): their descriptors (by slot),
    // their row-major tiles (anchors), the blocks of the tile and row-sum kernels
    SymPass *ddesc = nullptr;
    Tile *dtiles16 = nullptr;
    size_t tiles16_cap = 0;
    int *dstarts16 = nullptr;
    size_t starts16_cap = 0;
    std::vector<int> starts16_host;
    int2 *dwork = nullptr;
    size_t work_cap = 0;
    std::vector<int2> work_host;
    Sym16Launch s16{};
    bool has16 = false;
};

// ---------------------------------------------------------------------------------------

extern "C" {

const char *qcqp_last_error(void) { return g_err.c_str(); }

void qcqp_options_default(qcqp_options *o)
{
    std::memset(o, 0, sizeof(*o));
    o->variant = QCQP_YX;
    o->c_nm = 1;
    o->eta = 0.7;
    o->tau_bar = 0.0;
    o->gamma0 = 0.1;
    o->mu = 0.0;
    o->c_alpha = 0.4;
    o->c_beta = 0.0;
    o->delta = 0.5;
    o->restart = QCQP_RESTART_FIXED;
    o->restart_every = 400;
    o->restart_from_average = 0;
    o->xi = 0.04;
    o->q_restart = 0.5;
    o->ada_first = 50;
    o->ada_every = 500;
    o->max_iter = 50000;
    o->tol = 1e-6;
    o->storage = QCQP_F64;
    o->pass_mode = QCQP_PASS_AUTO;
    o->spec_trials = 2;
    o->poll_every = 0;
    o->timing = 0;
    o->inner_tol = 1e-12;
    o->max_inner = 100000;
    o->use_graphs = 1;
    o->stream = nullptr;
    o->stop_rule = QCQP_STOP_KKT;
    o->f_star = 0.0;
    o->sym_pass = 0;
}

static qcqp_status validate_options(const qcqp_options *o)
{
    if (o->variant != QCQP_YX && o->variant != QCQP_XY)
        return fail(QCQP_E_INVALID, "unknown variant %d", (int)o->variant);
    if (!(o->eta > 0.0 && o->eta < 1.0)) return fail(QCQP_E_INVALID, "eta must lie in (0,1)");
    if (!(o->gamma0 > 0.0) || !std::isfinite(o->gamma0)) return fail(QCQP_E_INVALID, "gamma0 must be > 0");
    if (!(o->tau_bar >= 0.0) || !std::isfinite(o->tau_bar)) return fail(QCQP_E_INVALID, "tau_bar must be >= 0");
    if (!(o->mu >= 0.0)) return fail(QCQP_E_INVALID, "mu must be >= 0");
    if (o->variant == QCQP_YX &&
        !(o->c_alpha > 0.0 && o->delta >= 0.0 && o->delta < 1.0 && o->c_alpha + o->delta <= 1.0))
        return fail(QCQP_E_INVALID, "APDB-yx needs c_alpha > 0, delta in [0,1), c_alpha + delta <= 1");
    // Algorithm 1 admits c_alpha, c_beta >= 0; a zero one divides a generally nonzero squared
    // gradient difference by alpha = 0 or beta = 0, and no trial could pass
    if (o->variant == QCQP_XY &&
        !(o->c_alpha > 0.0 && o->c_beta > 0.0 && o->delta >= 0.0 && o->c_alpha + o->c_beta + o->delta < 1.0))
        return fail(QCQP_E_INVALID, "APDB-xy needs c_alpha > 0, c_beta > 0, delta >= 0, c_alpha + c_beta + delta < 1");
    if (o->c_nm != 0 && o->c_nm != 1) return fail(QCQP_E_INVALID, "c_nm must be 0 or 1");
    if (o->restart < QCQP_RESTART_NONE || o->restart > QCQP_RESTART_ADAPTIVE)
        return fail(QCQP_E_INVALID, "unknown restart mode");
    if (o->restart == QCQP_RESTART_FIXED && o->restart_every < 1)
        return fail(QCQP_E_INVALID, "restart_every must be >= 1");
    if (o->restart == QCQP_RESTART_ADAPTIVE &&
        (o->ada_every < 1 || o->ada_first < 0 || !(o->xi > 0.0) || !(o->q_restart > 0.0 && o->q_restart < 1.0)))
        return fail(QCQP_E_INVALID, "adaptive restart needs ada_every >= 1, xi > 0, q in (0,1)");
    if (o->max_iter < 0) return fail(QCQP_E_INVALID, "max_iter must be >= 0");
    if (!(o->tol >= 0.0)) return fail(QCQP_E_INVALID, "tol must be >= 0");
    if (o->storage < QCQP_F64 || o->storage > QCQP_F16) return fail(QCQP_E_INVALID, "unknown storage type");
    if (o->stop_rule != QCQP_STOP_KKT && o->stop_rule != QCQP_STOP_PAPER)
        return fail(QCQP_E_INVALID, "unknown stop rule");
    if (o->stop_rule == QCQP_STOP_PAPER && !std::isfinite(o->f_star))
        return fail(QCQP_E_INVALID, "the PAPER stop rule needs a finite f_star");
    if (o->spec_trials < 1 || o->spec_trials > MAXB)
        return fail(QCQP_E_INVALID, "spec_trials must be in 1..%d", MAXB);
    if (o->pass_mode < QCQP_PASS_AUTO || o->pass_mode > QCQP_PASS_INCREMENTAL)
        return fail(QCQP_E_INVALID, "unknown pass mode");
    if (o->sym_pass != 0 && o->sym_pass != 1) return fail(QCQP_E_INVALID, "sym_pass must be 0 or 1");
    if (o->sym_pass && o->storage == QCQP_F64 && o->pass_mode == QCQP_PASS_INCREMENTAL)
        return fail(QCQP_E_INVALID, "sym_pass with F64 storage needs direct passes");
    if (o->sym_pass && (o->storage == QCQP_F32 || (o->storage != QCQP_F64 && o->pass_mode == QCQP_PASS_DIRECT)))
        return fail(QCQP_E_INVALID, "sym_pass needs F64 storage, or BF16/F16 storage with incremental passes");
    return QCQP_OK;
}

static void free_handle_memory(qcqp_handle *h)
{
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    h->ev_join = nullptr;
    if (h->stream) (void)hipStreamDestroy(h->stream);
    h->stream = nullptr;
    if (h->dQ) (void)hipFree(h->dQ);
    if (h->arena) (void)hipFree(h->arena);
    if (h->h_poll) (void)hipHostFree(h->h_poll);
    for (auto &x : h->ev_snap) {
        if (x) (void)hipEventDestroy(x);
        x = nullptr;
    }
    if (h->h_out) (void)hipHostFree(h->h_out);
    if (h->gap_mem) (void)hipFree(h->gap_mem);
    h->gap_mem = nullptr;
    if (h->dP) (void)hipFree(h->dP);
    if (h->dws) (void)hipFree(h->dws);
    if (h->dubase) (void)hipFree(h->dubase);
    if (h->dsym) (void)hipFree(h->dsym);
    h->dP = h->dws = nullptr;
    h->dubase = nullptr;
    h->dsym = nullptr;
    h->dQ = nullptr;
    h->arena = nullptr;
    h->h_poll = nullptr;
    h->h_out = nullptr;
}

// largest eigenvalue estimate of stored matrix `mat` by 30 power iterations from 1/sqrt(n),
// all on the device (the normalisation is a one-block kernel); one synchronisation at the end
static qcqp_status power_norm(qcqp_handle *h, int mat, double *out)
{
    const int64_t n = h->n;
    double *v = h->d_xe, *z = h->d_grad;
    HIPCHK(launch_fill(h->stream, v, n, 1.0 / std::sqrt((double)n)));
    for (int it = 0; it < 30; ++it) {
        HIPCHK(launch_matvec1(h->stream, h->dQ, h->dtype, (int)n, (int)h->ld, (int)(mat * n), v,
                              (int)h->nw, z));
        HIPCHK(launch_pow_normalize(h->stream, z, (int)n, v, h->d_out6));
    }
    HIPCHK(hipMemcpyAsync(h->h_out, h->d_out6, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    *out = h->h_out[0];
    return QCQP_OK;
}

qcqp_status qcqp_create(const qcqp_problem *P, const qcqp_options *opt, qcqp_handle **out)
{
    g_err.clear();
    if (!P || !out) return fail(QCQP_E_INVALID, "null argument");
    qcqp_options o;
    if (opt) o = *opt;
    else qcqp_options_default(&o);
    qcqp_status st = validate_options(&o);
    if (st) return st;
    const int64_t n = P->n, m = P->m, p = P->p;
    if (n <= 0 || m < 0 || p < 0 || p >= n) return fail(QCQP_E_INVALID, "need n > 0, m >= 0, 0 <= p < n");
    if (n > 16384 || m > 1024 || p > 64)
        return fail(QCQP_E_INVALID, "sizes beyond the supported limits (n<=16384, m<=1024, p<=64)");
    const int64_t ldq = P->ldq ? P->ldq : n;
    if (ldq < n) return fail(QCQP_E_INVALID, "ldq < n");
    if (!P->q || !P->c || !P->lb || !P->ub) return fail(QCQP_E_INVALID, "q, c, lb, ub are required");
    if (p > 0 && (!P->A || !P->b)) return fail(QCQP_E_INVALID, "A and b are required when p > 0");
    if (P->q_stored) {
        if ((P->q_stored[0] != 0) != (P->has_q0 != 0))
            return fail(QCQP_E_INVALID, "q_stored[0] must equal has_q0");
        for (int64_t i = 0; i <= m; ++i)
            if (P->q_stored[i] != 0 && P->q_stored[i] != 1) return fail(QCQP_E_INVALID, "q_stored flags must be 0 or 1");
    }
    int64_t nstored = 0;
    for (int64_t i = 0; i <= m; ++i)
        nstored += P->q_stored ? P->q_stored[i] : (i == 0 ? (P->has_q0 ? 1 : 0) : 1);
    if (nstored > 0 && !P->Q) return fail(QCQP_E_INVALID, "Q is required");
    if (P->lambda_set == QCQP_LAMBDA_CONES) {
        if (P->n_soc < 1 || !P->soc_dims) return fail(QCQP_E_INVALID, "CONES needs n_soc >= 1 and soc_dims");
        int64_t tot = 0;
        for (int64_t c = 0; c < P->n_soc; ++c) {
            if (P->soc_dims[c] < 1) return fail(QCQP_E_INVALID, "cone dimensions must be >= 1");
            tot += P->soc_dims[c];
        }
        if (tot > m) return fail(QCQP_E_INVALID, "cone dimensions sum to %lld > m", (long long)tot);
    }
    if (P->Q_dtype < QCQP_F64 || P->Q_dtype > QCQP_F16) return fail(QCQP_E_INVALID, "unknown Q_dtype");
    if (P->lambda_set != QCQP_LAMBDA_NONNEG && P->lambda_set != QCQP_LAMBDA_SIMPLEX &&
        P->lambda_set != QCQP_LAMBDA_CONES)
        return fail(QCQP_E_INVALID, "unknown lambda_set");
    if (P->lambda_set == QCQP_LAMBDA_SIMPLEX && m < 1) return fail(QCQP_E_INVALID, "the simplex needs m >= 1");
    if (!(P->q0_shift >= 0.0) || !std::isfinite(P->q0_shift)) return fail(QCQP_E_INVALID, "q0_shift must be finite and >= 0");
    if (!(P->ball >= 0.0 && P->ball_v >= 0.0 && P->ball_lambda >= 0.0) ||
        !std::isfinite(P->ball) || !std::isfinite(P->ball_v) || !std::isfinite(P->ball_lambda))
        return fail(QCQP_E_INVALID, "ball radii must be finite and >= 0");
    if (P->ball > 0.0 && (P->ball_v > 0.0 || P->ball_lambda > 0.0))
        return fail(QCQP_E_INVALID, "use either the joint ball or the separable balls");
    // the simplex is compact already and not a cone: a ball on lambda would need another projection
    if (P->lambda_set == QCQP_LAMBDA_SIMPLEX && (P->ball > 0.0 || P->ball_lambda > 0.0))
        return fail(QCQP_E_INVALID, "with the simplex only the ball on v is supported");
    const int has_q0 = P->has_q0 ? 1 : 0;
    const int64_t nq = nstored;
    // position of Q_i among the stored matrices (-1: Q_i = 0, not stored)
    std::vector<int32_t> qmap(m + 1, -1);
    {
        int32_t sidx = 0;
        for (int64_t i = 0; i <= m; ++i)
            if (P->q_stored ? P->q_stored[i] != 0 : (i > 0 || has_q0)) qmap[i] = sidx++;
    }
    // cone tables: start offsets within lambda, dimensions, and the large cones
    std::vector<int32_t> soc_tab, soc_big;
    int64_t m0 = m;
    if (P->lambda_set == QCQP_LAMBDA_CONES) {
        for (int64_t c = 0; c < P->n_soc; ++c) m0 -= P->soc_dims[c];
        soc_tab.resize(2 * P->n_soc);
        int64_t off = m0;
        for (int64_t c = 0; c < P->n_soc; ++c) {
            soc_tab[c] = (int32_t)off;
            soc_tab[P->n_soc + c] = (int32_t)P->soc_dims[c];
            if (P->soc_dims[c] >= SOC_BLOCK_DIM) soc_big.push_back((int32_t)c);
            off += P->soc_dims[c];
        }
    }

    qcqp_handle *h = new (std::nothrow) qcqp_handle();
    if (!h) return fail(QCQP_E_NOMEM, "host allocation");
    h->opt = o;
    h->n = n; h->m = m; h->p = p; h->ny = p + m; h->nq = nq; h->has_q0 = has_q0;
    h->on_device = P->on_device ? 1 : 0;
    h->dtype = (int)o.storage;
    h->ustream = (hipStream_t)o.stream;
    h->B = o.spec_trials;
    h->incremental = o.pass_mode == QCQP_PASS_INCREMENTAL ||
                     (o.pass_mode == QCQP_PASS_AUTO && o.storage != QCQP_F64);
    if (hipGetDevice(&h->dev) != hipSuccess) { delete h; return fail(QCQP_E_DEVICE, "no HIP device"); }
    if ((st = ensure_prepared())) { delete h; return st; }
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess) {
        if (h->stream) (void)hipStreamDestroy(h->stream);
        delete h;
        return fail(QCQP_E_DEVICE, "stream creation");
    }
    // inputs written on the caller's stream are complete before the library reads them
    if (hipEventRecord(h->ev_join, h->ustream) != hipSuccess ||
        hipStreamWaitEvent(h->stream, h->ev_join, 0) != hipSuccess) {
        (void)hipStreamDestroy(h->stream);
        (void)hipEventDestroy(h->ev_join);
        delete h;
        return fail(QCQP_E_DEVICE, "stream join");
    }

    // ---- host-side validation of the small vectors (copied to host when on device) ----
    std::vector<double> hq((m + 1) * n), hc(m + 1), hlb(n), hub(n), hA(p * n), hb(p);
    auto fetch = [&](std::vector<double> &dst, const double *src, size_t cnt) -> qcqp_status {
        if (cnt == 0) return QCQP_OK;
        if (h->on_device) HIPCHK(hipMemcpy(dst.data(), src, cnt * sizeof(double), hipMemcpyDeviceToHost));
        else std::memcpy(dst.data(), src, cnt * sizeof(double));
        return QCQP_OK;
    };
    if ((st = fetch(hq, P->q, hq.size())) || (st = fetch(hc, P->c, hc.size())) ||
        (st = fetch(hlb, P->lb, n)) || (st = fetch(hub, P->ub, n)) ||
        (st = fetch(hA, P->A, hA.size())) || (st = fetch(hb, P->b, hb.size()))) {
        delete h;
        return st;
    }
    for (int64_t j = 0; j < n; ++j)
        if (!(hlb[j] <= hub[j]) || hlb[j] == INFINITY || hub[j] == -INFINITY) {
            delete h;
            return fail(QCQP_E_INVALID, "box bounds need lb <= ub, lb < +inf, ub > -inf (index %lld)",
                        (long long)j);
        }
    for (double v : hq) if (!std::isfinite(v)) { delete h; return fail(QCQP_E_INVALID, "non-finite q"); }
    for (double v : hc) if (!std::isfinite(v)) { delete h; return fail(QCQP_E_INVALID, "non-finite c"); }
    for (double v : hA) if (!std::isfinite(v)) { delete h; return fail(QCQP_E_INVALID, "non-finite A"); }
    for (double v : hb) if (!std::isfinite(v)) { delete h; return fail(QCQP_E_INVALID, "non-finite b"); }

    // ---- Q stack in the storage type, rows padded to 128 bytes ----
    const int es = elem_size(h->dtype);
    h->ld = round_up(n, 128 / es);
    h->nw = round_up(n, vec_width(h->dtype));
    {
        // the row-major trial pass stages B candidates in LDS; the packed symmetric pass keeps
        // them in registers, and only the single-vector products (step-size estimate) stage x
        const size_t acc = h->dtype == DT_F64 ? 8 : 4;
        const size_t trial = o.sym_pass ? 0 : (size_t)h->B * h->nw * acc;
        const size_t lds = std::max<size_t>((size_t)h->nw * 8, trial);
        if (lds > (size_t)max_lds) {
            delete h;
            return fail(QCQP_E_INVALID, "n = %lld with spec_trials = %d needs %zu bytes of LDS (device allows %d)",
                        (long long)n, o.spec_trials, lds, max_lds);
        }
    }
    h->q_bytes = (size_t)nq * n * h->ld * es;
    // three words per stored matrix for the symmetry check, after the stack
    const size_t chk_bytes = (size_t)round_up(3 * nq * (int64_t)sizeof(unsigned long long), 256);
    if (nq > 0) {
        if (hipMalloc(&h->dQ, h->q_bytes + chk_bytes) != hipSuccess) {
            delete h;
            return fail(QCQP_E_NOMEM, "Q stack (%zu bytes)", h->q_bytes);
        }
        const int sdt = (int)P->Q_dtype;
        const size_t smat = (size_t)n * ldq * elem_size(sdt);
        void *stage = nullptr;
        if (sdt == h->dtype) {
            // same element type: one pitched copy of the whole stack (the stored rows are
            // padded to ld), and the padding columns cleared
            hipError_t e = hipMemcpy2DAsync(h->dQ, (size_t)h->ld * es, P->Q, (size_t)ldq * es, (size_t)n * es,
                                            (size_t)nq * n, h->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                            h->stream);
            if (e == hipSuccess && h->ld > n)
                e = hipMemset2DAsync((char *)h->dQ + (size_t)n * es, (size_t)h->ld * es, 0, (size_t)(h->ld - n) * es,
                                     (size_t)nq * n, h->stream);
            if (e != hipSuccess) {
                free_handle_memory(h);
                delete h;
                return fail(QCQP_E_DEVICE, "Q upload: %s", hipGetErrorString(e));
            }
        } else {
        if (!h->on_device) {
            if (hipMalloc(&stage, smat) != hipSuccess) {
                free_handle_memory(h);
                delete h;
                return fail(QCQP_E_NOMEM, "staging buffer");
            }
        }
        for (int64_t i = 0; i < nq; ++i) {
            const char *src = (const char *)P->Q + i * smat;
            const void *dsrc = src;
            hipError_t e = hipSuccess;
            if (!h->on_device) {
                e = hipMemcpy(stage, src, smat, hipMemcpyHostToDevice);
                dsrc = stage;
            }
            if (e == hipSuccess)
                e = launch_convert(h->stream, dsrc, sdt, ldq, (char *)h->dQ + (size_t)i * n * h->ld * es,
                                   h->dtype, h->ld, n, n);
            if (e == hipSuccess && !h->on_device) e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) {
                if (stage) (void)hipFree(stage);
                free_handle_memory(h);
                delete h;
                return fail(QCQP_E_DEVICE, "Q upload/convert: %s", hipGetErrorString(e));
            }
        }
        }
        if (stage) (void)hipFree(stage);
        // the stored matrices must be finite and symmetric
        unsigned long long *dchk = (unsigned long long *)((char *)h->dQ + h->q_bytes);
        std::vector<unsigned long long> chk(3 * nq, 0ull);
        hipError_t e = hipMemsetAsync(dchk, 0, chk.size() * sizeof(unsigned long long), h->stream);
        if (e == hipSuccess) e = launch_sym_check(h->stream, h->dQ, h->dtype, h->ld, (int)n, (int)nq, dchk);
        if (e == hipSuccess)
            e = hipMemcpyAsync(chk.data(), dchk, chk.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) {
            free_handle_memory(h);
            delete h;
            return fail(QCQP_E_DEVICE, "Q symmetry check: %s", hipGetErrorString(e));
        }
        for (int64_t i = 0; i < nq; ++i) {
            const double dmax = __builtin_bit_cast(double, (uint64_t)chk[3 * i]);
            const double amax = __builtin_bit_cast(double, (uint64_t)chk[3 * i + 1]);
            if (chk[3 * i + 2]) {
                free_handle_memory(h);
                delete h;
                return fail(QCQP_E_INVALID, "stored matrix %lld of Q has a non-finite entry", (long long)i);
            }
            if (dmax > SYMMETRY_TOL * amax) {
                free_handle_memory(h);
                delete h;
                return fail(QCQP_E_INVALID,
                            "stored matrix %lld of Q is not symmetric: max |Q_rc - Q_cr| = %.3g > %.0e max |Q_rc| = %.3g",
                            (long long)i, dmax, SYMMETRY_TOL, SYMMETRY_TOL * amax);
            }
        }
    }

    // ---- options.sym_pass: the packed upper-triangle copy of the stack ----
    if (o.sym_pass && nq > 0 && h->dtype != DT_F64) {
        // 16-bit storage: SYM16_T-wide tiles of the stored values, FP32 per-tile results
        const int32_t NT = (int32_t)((n + SYM16_T - 1) / SYM16_T);
        const int64_t ntt = (int64_t)NT * (NT + 1) / 2;
        const size_t pbytes = (size_t)nq * ntt * SYM16_TILE * 2;
        const size_t wbytes = (size_t)nq * ntt * 2 * h->B * SYM16_T * sizeof(float);
        std::vector<int32_t> ub;
        for (int64_t i = 0; i <= m; ++i)
            if (qmap[i] >= 0) ub.push_back((int32_t)(i * n));
        const size_t nub = ub.size();
        ub.push_back(0);   // the packing's inexact-halving flag
        if (hipMalloc(&h->dP, pbytes) != hipSuccess || hipMalloc(&h->dws, wbytes) != hipSuccess ||
            hipMalloc(&h->dubase, ub.size() * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&h->dsym, sizeof(SymPass)) != hipSuccess) {
            free_handle_memory(h);
            delete h;
            return fail(QCQP_E_NOMEM, "packed symmetric stack (%zu bytes)", pbytes + wbytes);
        }
        h->sym = SymPass{nullptr, nullptr, h->dubase, (int32_t)n, NT, (int32_t)ntt, (int32_t)nq, (int32_t)h->B,
                         h->dtype, reinterpret_cast<const uint16_t *>(h->dP), reinterpret_cast<float *>(h->dws)};
        h->s16 = Sym16Launch{h->dtype, h->B, h->dsym, nullptr, (int32_t)(nq * ntt), nullptr, (int32_t)(nq * NT),
                             nullptr, 0, 0, nullptr};
        unsigned *inexact = reinterpret_cast<unsigned *>(h->dubase + nub);
        unsigned flag = 0;
        hipError_t e = hipMemcpyAsync(h->dubase, ub.data(), ub.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                      h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(h->dsym, &h->sym, sizeof(SymPass), hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = launch_sym_pack16(h->stream, h->dQ, h->ld, h->dtype, h->sym, h->dP, inexact);
        if (e == hipSuccess) e = hipMemcpyAsync(&flag, inexact, sizeof(flag), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);   // ub is read by the copy
        if (e != hipSuccess) {
            free_handle_memory(h);
            delete h;
            return fail(QCQP_E_DEVICE, "packing the symmetric stack: %s", hipGetErrorString(e));
        }
        if (flag) {
            free_handle_memory(h);
            delete h;
            return fail(QCQP_E_INVALID, "sym_pass: a diagonal entry of Q is too small to halve exactly in the storage type");
        }
        h->use_sym = true;
        h->sym_bytes = pbytes + wbytes + ub.size() * sizeof(int32_t) + sizeof(SymPass);
    } else if (o.sym_pass && nq > 0) {
        const int32_t NT = (int32_t)((n + SYM_T - 1) / SYM_T);
        const int64_t ntt = (int64_t)NT * (NT + 1) / 2;
        const size_t pbytes = (size_t)nq * ntt * SYM_TILE_STRIDE * sizeof(double);
        const size_t wbytes = (size_t)nq * ntt * 2 * h->B * SYM_T * sizeof(double);
        std::vector<int32_t> ub;
        for (int64_t i = 0; i <= m; ++i)
            if (qmap[i] >= 0) ub.push_back((int32_t)(i * n));
        if (hipMalloc(&h->dP, pbytes) != hipSuccess || hipMalloc(&h->dws, wbytes) != hipSuccess ||
            hipMalloc(&h->dubase, ub.size() * sizeof(int32_t)) != hipSuccess) {
            free_handle_memory(h);
            delete h;
            return fail(QCQP_E_NOMEM, "packed symmetric stack (%zu bytes)", pbytes + wbytes);
        }
        h->sym = SymPass{h->dP, h->dws, h->dubase, (int32_t)n, NT, (int32_t)ntt, (int32_t)nq, (int32_t)h->B,
                         DT_F64, nullptr, nullptr};
        hipError_t e = hipMemcpyAsync(h->dubase, ub.data(), ub.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                      h->stream);
        if (e == hipSuccess) e = launch_sym_pack(h->stream, (const double *)h->dQ, h->ld, h->sym, h->dP);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);   // ub is read by the copy
        if (e != hipSuccess) {
            free_handle_memory(h);
            delete h;
            return fail(QCQP_E_DEVICE, "packing the symmetric stack: %s", hipGetErrorString(e));
        }
        h->use_sym = true;
        h->sym_bytes = pbytes + wbytes + ub.size() * sizeof(int32_t);
    }

    // ---- arena for vectors and state ----
    const int B = h->B;
    h->nblk_step = (int)((n + STEP_COLS - 1) / STEP_COLS);
    const int64_t ny = h->ny, U1 = (m + 1) * n;
    std::vector<std::pair<double **, int64_t>> plan;
    Slot &S = h->hslot;
    std::memset(&S, 0, sizeof(S));
    double *dq, *dc, *dA = nullptr, *db = nullptr, *dlb, *dub;
    plan.push_back({&dq, U1});
    plan.push_back({&dc, m + 1});
    if (p) { plan.push_back({&dA, p * n}); plan.push_back({&db, p}); }
    plan.push_back({&dlb, n});
    plan.push_back({&dub, n});
    plan.push_back({&S.x, n});
    for (int b = 0; b < B; ++b) plan.push_back({&S.xc[b], n});
    plan.push_back({&S.U, U1});
    for (int b = 0; b < B; ++b) plan.push_back({&S.Uc[b], U1});
    if (h->incremental)
        for (int b = 0; b < B; ++b) plan.push_back({&S.W[b], U1});
    plan.push_back({&S.y, ny + 1});
    for (int b = 0; b < B; ++b) plan.push_back({&S.yc[b], ny + 1});
    plan.push_back({&S.G, ny + 1});
    for (int b = 0; b < B; ++b) plan.push_back({&S.Gc[b], ny + 1});
    plan.push_back({&S.Gp, ny + 1});
    for (int b = 0; b < B; ++b) plan.push_back({&S.dG[b], ny + 1});
    plan.push_back({&S.e, MAXB * (m + 1)});
    plan.push_back({&S.cx, n});
    plan.push_back({&S.cy, ny + 1});
    plan.push_back({&S.part, (int64_t)h->nblk_step * NPART});
    if (o.variant == QCQP_XY) {
        plan.push_back({&S.gxk, n});
        plan.push_back({&S.gxp, n});
        plan.push_back({&S.part2, (int64_t)h->nblk_step * NPART2});
    }
    plan.push_back({&h->d_ueval, U1});
    plan.push_back({&h->d_geval, ny + 1});
    plan.push_back({&h->d_grad, n});
    plan.push_back({&h->d_kpart, (int64_t)h->nblk_step * 4});
    plan.push_back({&h->d_out6, 8});
    plan.push_back({&h->d_xe, n});
    plan.push_back({&h->d_ye, ny + 1});
    // int32 tables, each in whole doubles: the stored-matrix map and the cone tables
    double *d_qmap = nullptr, *d_soc = nullptr, *d_socbig = nullptr;
    plan.push_back({&d_qmap, (m + 2) / 2});
    if (!soc_tab.empty()) plan.push_back({&d_soc, ((int64_t)soc_tab.size() + 1) / 2});
    if (!soc_big.empty()) plan.push_back({&d_socbig, ((int64_t)soc_big.size() + 1) / 2});
    size_t total = 0;
    for (auto &pr : plan) total += (size_t)round_up(pr.second * 8, 256);
    const size_t slot_off = total;
    total += 2 * round_up(sizeof(Slot), 256);
    const size_t live_off = total;
    total += 256;
    // tiles
    int lpr = 16, rpt = 16;
    tile_shape(n, h->dtype, nq * n, &lpr, &rpt);
    const int64_t rows = nq * n;
    (void)rows;
    // Tiles cover runs of consecutive stored matrices whose rows of U are consecutive too (the
    // whole stack for a plain QCQP); each carries the offset from its stored rows to the rows
    // of U it produces (Q_i stored s-th writes U_i).
    for (int64_t i = 0; i <= m;) {
        if (qmap[i] < 0) {
            ++i;
            continue;
        }
        int64_t j = i;
        while (j + 1 <= m && qmap[j + 1] == qmap[j] + 1) ++j;
        const int64_t sbase = (int64_t)qmap[i] * n, run = (j - i + 1) * n;
        const int32_t uoff = (int32_t)((i - qmap[i]) * n);
        for (int64_t r0 = 0; r0 < run; r0 += rpt)
            h->tiles.push_back(Tile{0, (int32_t)(sbase + r0), (int32_t)std::min<int64_t>(rpt, run - r0), lpr, uoff});
        i = j + 1;
    }
    const size_t tile_off = total;
    total += round_up((int64_t)std::max<size_t>(h->tiles.size(), 1) * sizeof(Tile), 256);
    const size_t starts_off = total;
    total += round_up((int64_t)(h->tiles.size() + 2) * sizeof(int), 256);
    h->pass_grid = pass_grid_for(B, h->dtype, (int)h->nw, (double)h->q_bytes);
    h->nt = (double)h->q_bytes > CACHE_RESIDENT_BYTES ? 1 : 0;
    if (hipMalloc(&h->arena, total) != hipSuccess) {
        free_handle_memory(h);
        delete h;
        return fail(QCQP_E_NOMEM, "state arena (%zu bytes)", total);
    }
    h->arena_bytes = total;
    {
        size_t off = 0;
        for (auto &pr : plan) {
            *pr.first = reinterpret_cast<double *>(h->arena + off);
            off += (size_t)round_up(pr.second * 8, 256);
        }
    }
    h->dslot = reinterpret_cast<Slot *>(h->arena + slot_off);
    h->dslot_eval = reinterpret_cast<Slot *>(h->arena + slot_off + round_up(sizeof(Slot), 256));
    h->dlive0 = reinterpret_cast<int *>(h->arena + live_off);
    h->dtiles = reinterpret_cast<Tile *>(h->arena + tile_off);
    h->dstarts = reinterpret_cast<int *>(h->arena + starts_off);
    hipError_t e = hipMemsetAsync(h->arena, 0, total, h->stream);
    if (e == hipSuccess && !h->tiles.empty())
        e = hipMemcpyAsync(h->dtiles, h->tiles.data(), h->tiles.size() * sizeof(Tile),
                           hipMemcpyHostToDevice, h->stream);
    // the pass launch clips its grid to max(1, min(pass_grid, tiles)); the table matches it
    std::vector<int> hstarts;
    {
        std::vector<int64_t> tb;
        for (const Tile &t : h->tiles) tb.push_back((int64_t)t.nrows * n * es);
        hstarts = balanced_starts(tb, std::max(1, std::min<int>(h->pass_grid, (int)h->tiles.size())));
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->dstarts, hstarts.data(), hstarts.size() * sizeof(int), hipMemcpyHostToDevice,
                               h->stream);
    }
    const hipMemcpyKind k = hipMemcpyHostToDevice;
    if (e == hipSuccess) e = hipMemcpyAsync(dq, hq.data(), U1 * 8, k, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dc, hc.data(), (m + 1) * 8, k, h->stream);
    if (e == hipSuccess && p) e = hipMemcpyAsync(dA, hA.data(), p * n * 8, k, h->stream);
    if (e == hipSuccess && p) e = hipMemcpyAsync(db, hb.data(), p * 8, k, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_qmap, qmap.data(), (m + 1) * sizeof(int32_t), k, h->stream);
    if (e == hipSuccess && d_soc)
        e = hipMemcpyAsync(d_soc, soc_tab.data(), soc_tab.size() * sizeof(int32_t), k, h->stream);
    if (e == hipSuccess && d_socbig)
        e = hipMemcpyAsync(d_socbig, soc_big.data(), soc_big.size() * sizeof(int32_t), k, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dlb, hlb.data(), n * 8, k, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dub, hub.data(), n * 8, k, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipHostMalloc((void **)&h->h_poll, 2 * sizeof(Slot));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_snap[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_snap[1], hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void **)&h->h_out, 16 * sizeof(double));
    if (e != hipSuccess) {
        free_handle_memory(h);
        delete h;
        return fail(QCQP_E_DEVICE, "initial upload: %s", hipGetErrorString(e));
    }

    // ---- constant slot fields ----
    S.n = (int32_t)n; S.m = (int32_t)m; S.p = (int32_t)p; S.ny = (int32_t)ny;
    S.nq = (int32_t)nq; S.has_q0 = has_q0; S.ld = (int32_t)h->ld; S.dtype = h->dtype;
    S.c_nm = o.c_nm; S.restart = (int32_t)o.restart; S.restart_from_avg = o.restart_from_average ? 1 : 0;
    S.incremental = h->incremental; S.B = B; S.nblk_step = h->nblk_step; S.nw = (int32_t)h->nw;
    S.variant = o.variant == QCQP_XY ? VAR_XY : VAR_YX;
    S.q0_shift = P->q0_shift;
    S.n_soc = (int32_t)(P->lambda_set == QCQP_LAMBDA_CONES ? P->n_soc : 0);
    S.m0 = (int32_t)m0;
    S.n_soc_big = (int32_t)soc_big.size();
    S.soc_off = reinterpret_cast<const int32_t *>(d_soc);
    S.soc_big = reinterpret_cast<const int32_t *>(d_socbig);
    S.qmap = reinterpret_cast<const int32_t *>(d_qmap);
    S.lambda_set = P->lambda_set == QCQP_LAMBDA_SIMPLEX ? LAMBDA_SIMPLEX
                   : (P->lambda_set == QCQP_LAMBDA_CONES ? LAMBDA_CONES : LAMBDA_NONNEG);
    S.ball = P->ball;
    S.ball_v = P->ball_v;
    S.ball_l = P->ball_lambda;
    S.restart_every = o.restart_every; S.ada_first = o.ada_first; S.ada_every = o.ada_every;
    S.max_iter = o.max_iter;
    S.eta = o.eta; S.gamma0 = o.gamma0; S.mu = o.mu; S.c_alpha = o.c_alpha; S.c_beta = o.c_beta;
    S.delta = o.delta;
    S.tol = o.tol; S.q_restart = o.q_restart;
    S.stop_rule = o.stop_rule == QCQP_STOP_PAPER ? 1 : 0;
    S.f_star = o.f_star;
    double cn = 0.0, bn = 0.0;
    for (int64_t i = 1; i <= m; ++i) cn += hc[i] * hc[i];
    for (int64_t l = 0; l < p; ++l) bn += hb[l] * hb[l];
    S.cnorm = std::sqrt(cn);
    S.bnorm = std::sqrt(bn);
    S.Q = h->dQ; S.q = dq; S.c = dc; S.A = dA; S.b = db; S.lb = dlb; S.ub = dub;

    // ---- default initial step: 1 / ||Q_0 + rho I||_2 (or 1 / max_i ||Q_i||_2 when the
    //      objective has no quadratic part) ----
    double tau_bar = o.tau_bar;
    if (!(tau_bar > 0.0)) {
        double L = 0.0;
        if (has_q0 || P->q0_shift > 0.0) {
            if (has_q0 && (st = power_norm(h, 0, &L))) { free_handle_memory(h); delete h; return st; }
            L += P->q0_shift;     // Q_0 is positive semidefinite
        } else {
            for (int mat = 0; mat < (int)nq; ++mat) {
                double lm = 0.0;
                if ((st = power_norm(h, mat, &lm))) { free_handle_memory(h); delete h; return st; }
                L = std::max(L, lm);
            }
        }
        tau_bar = L > 0.0 ? 1.0 / L : 1.0;
    }
    S.tau_bar = tau_bar;
    h->opt.tau_bar = tau_bar;
    *out = h;
    return QCQP_OK;
}

size_t qcqp_handle_bytes(const qcqp_handle *h) { return h ? h->q_bytes + h->arena_bytes + h->sym_bytes : 0; }

qcqp_status qcqp_destroy(qcqp_handle *h)
{
    if (!h) return QCQP_OK;
    if (h->owner) return fail(QCQP_E_INVALID, "handle is admitted to a batch; fetch it first");
    free_handle_memory(h);
    delete h;
    return QCQP_OK;
}

// ---------------------------------------------------------------------------------------
// run-state helpers

static void reset_run_scalars(Slot &S)
{
    S.tau = S.tau_bar;
    S.tau_prev = S.tau_bar;
    S.sig_prev = S.gamma0 * S.tau_bar;
    S.gam = S.gamma0;
    S.sig0 = 0.0;
    // alpha_0, beta_0 from tau_{-1}, sigma_{-1} (Algorithm 1, first line)
    S.alpha_k = S.c_alpha / (S.variant == VAR_XY ? S.tau_prev : S.sig_prev);
    S.beta_k = S.gamma0 * S.c_beta / S.sig_prev;
    S.T = 0.0;
    for (double &v : S.kkt) v = NAN;
    S.crit = NAN;
    S.f = NAN;
    S.maxviol = NAN;
    S.Gref = NAN;
    S.last_gap = NAN;
    S.k = S.ke = S.trials = S.passes = S.restarts = S.gap_evals = S.iter_trials = 0;
    S.status = ST_RUNNING;
    S.mode = MODE_ANCHOR;
    S.fresh = 0;
    S.anchor_keep_gp = 0;
}

// copy x0 (or zeros) and y0 (or zeros) into the canonical iterate buffers
static qcqp_status load_start(qcqp_handle *h, const double *x0, const double *y0)
{
    const hipMemcpyKind k = h->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (x0) HIPCHK(hipMemcpyAsync(h->hslot.x, x0, h->n * 8, k, h->stream));
    else HIPCHK(hipMemsetAsync(h->hslot.x, 0, h->n * 8, h->stream));
    if (h->ny) {
        if (y0) HIPCHK(hipMemcpyAsync(h->hslot.y, y0, h->ny * 8, k, h->stream));
        else HIPCHK(hipMemsetAsync(h->hslot.y, 0, h->ny * 8, h->stream));
    }
    return QCQP_OK;
}

static void fill_info(const qcqp_handle *h, const Slot &S, qcqp_info *info, double secs,
                      double pass_secs, int64_t timed)
{
    if (!info) return;
    std::memset(info, 0, sizeof(*info));
    info->iters = S.k;
    info->trials = S.trials;
    info->q_passes = S.passes;
    info->restarts = S.restarts;
    info->gap_evals = S.gap_evals;
    info->rel_kkt = S.kkt[0];
    info->rel_dual = S.kkt[1];
    info->rel_pri = S.kkt[2];
    info->rel_comp = S.kkt[3];
    info->f = S.f;
    info->max_violation = S.maxviol;
    info->seconds = secs;
    info->pass_seconds = pass_secs;
    info->timed_passes = timed;
    info->last_gap = S.last_gap;
    info->stop_value = S.crit;
    info->pass_bytes = h->use_sym ? (int64_t)h->nq * (h->n * (h->n + 1) / 2) * elem_size(h->dtype)
                                  : (int64_t)h->nq * h->n * h->n * elem_size(h->dtype);
    switch (S.status) {
    case ST_CONVERGED: info->status = QCQP_OK; break;
    case ST_MAX_ITER: info->status = QCQP_E_NOT_CONVERGED; break;
    case ST_NUMERICAL: info->status = QCQP_E_NUMERICAL; break;
    default: info->status = QCQP_E_NOT_CONVERGED; break;
    }
}

static qcqp_status slot_status_code(int st)
{
    switch (st) {
    case ST_CONVERGED: return QCQP_OK;
    case ST_MAX_ITER: return QCQP_E_NOT_CONVERGED;
    case ST_NUMERICAL: return fail(QCQP_E_NUMERICAL, "NaN/Inf met or the backtracking step underflowed");
    default: return QCQP_E_NOT_CONVERGED;
    }
}

static qcqp_status run_gap_for(qcqp_handle *h, Slot *dslot, const double *x_dev, const double *y_dev,
                               hipStream_t decide_stream);

qcqp_status qcqp_solve(qcqp_handle *h, const double *x0, const double *y0, double *x_out,
                       double *y_out, qcqp_info *info)
{
    g_err.clear();
    if (!h || !x_out) return fail(QCQP_E_INVALID, "null argument");
    if (h->owner) return fail(QCQP_E_INVALID, "handle is admitted to a batch");
    const double t0 = now_s();
    qcqp_status st;
    HIPCHK(join_streams(h->stream, h->ustream, h->ev_join));
    if ((st = load_start(h, x0, y0))) return st;
    Slot S0 = h->hslot;
    reset_run_scalars(S0);
    HIPCHK(hipMemcpyAsync(h->dslot, &S0, sizeof(Slot), hipMemcpyHostToDevice, h->stream));
    HIPCHK(launch_start(h->stream, h->dslot));
    int64_t poll = h->opt.poll_every;
    if (poll <= 0) {
        // about 1 ms of work per chunk, from the pass at ~5 TB/s plus ~40 us of small kernels
        const double group_s = (double)h->q_bytes / 5e12 + 40e-6;
        poll = std::max<int64_t>(4, (int64_t)std::ceil(1e-3 / group_s));
    }
    const bool timing = h->opt.timing != 0;
    // timing: two sets of per-group events, one per chunk of the pipelined polls below
    std::vector<hipEvent_t> ev;
    if (timing) {
        ev.resize(4 * poll);
        for (auto &x : ev) HIPCHK(hipEventCreate(&x));
    }
    double pass_secs = 0.0;
    int64_t timed = 0;
    const int ntiles = (int)h->tiles.size();
    Slot snap = S0;           // the last status snapshot read on the host
    qcqp_status result = QCQP_OK;
    int64_t passes_before = 0;
    auto launch_chunk = [&](hipStream_t s, bool with_events, int set = 0) -> hipError_t {
        for (int64_t g = 0; g < poll; ++g) {
            hipError_t e = launch_group(s, h->dslot, nullptr, 1, h->dtiles, ntiles, h->dstarts, h->B, h->dtype,
                                        h->hslot.variant == VAR_XY ? HAS_XY : HAS_YX, h->nblk_step, (int)std::max<int64_t>(h->ny, 1), (int)h->nw,
                                        (int)(h->m + 1 + h->p), h->pass_grid, h->nt,
                                        with_events ? ev[2 * (set * poll + g)] : nullptr,
                                        with_events ? ev[2 * (set * poll + g) + 1] : nullptr,
                                        h->sym64(), h->sym16());
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    const bool graphs = h->opt.use_graphs && !timing;
    if (graphs && (!h->gexec || h->gexec_groups != poll)) {
        if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
        HIPCHK(capture_graph(h->stream, [&](hipStream_t s) { return launch_chunk(s, false); }, &h->gexec));
        h->gexec_groups = poll;
    }
    // Pipelined polls: one chunk is always queued behind the one whose status snapshot the host
    // reads, so the device does not idle for the host round trip.  Once the slot stops running
    // every later group returns at once, so the extra chunk is a no-op; at a pending G_xi
    // evaluation the queue is drained first.  With timing, chunk buffer `buf` records its
    // groups' pass events in event set `buf`, read once its snapshot has arrived.
    {
        auto enqueue = [&](int buf) -> hipError_t {
            hipError_t e = graphs ? hipGraphLaunch(h->gexec, h->stream) : launch_chunk(h->stream, timing, buf);
            if (e == hipSuccess)
                e = hipMemcpyAsync(&h->h_poll[buf], h->dslot, sizeof(Slot), hipMemcpyDeviceToHost, h->stream);
            if (e == hipSuccess) e = hipEventRecord(h->ev_snap[buf], h->stream);
            return e;
        };
        int pending = 0;
        hipError_t e = enqueue(0);
        while (e == hipSuccess) {
            e = enqueue(1 - pending);
            if (e == hipSuccess) e = hipEventSynchronize(h->ev_snap[pending]);
            if (e != hipSuccess) break;
            const Slot &sn = h->h_poll[pending];
            if (timing) {
                // the groups that streamed a pass are the first (passes now - passes before) of
                // the chunk: once the slot stops running every later group is a no-op
                const int64_t worked = std::min<int64_t>(poll, sn.passes - passes_before);
                for (int64_t g = 0; g < worked; ++g) {
                    float ms = 0.f;
                    if (hipEventElapsedTime(&ms, ev[2 * (pending * poll + g)], ev[2 * (pending * poll + g) + 1]) ==
                        hipSuccess) {
                        pass_secs += ms * 1e-3;
                        timed += 1;
                    }
                }
                passes_before = sn.passes;
            }
            if (sn.status == ST_GAP_PENDING) {
                // the chunk queued behind this snapshot returns at once (the slot is not
                // running); G_xi and the decision follow it on the stream, then the next chunks
                snap = sn;
                if ((result = run_gap_for(h, h->dslot, sn.x, sn.y, h->stream))) break;
                pending = 0;
                e = enqueue(0);
                continue;
            }
            if (sn.status != ST_RUNNING) {
                e = hipStreamSynchronize(h->stream);
                snap = sn;
                break;
            }
            pending = 1 - pending;
        }
        if (e != hipSuccess && !result) result = fail(QCQP_E_DEVICE, "launch/poll: %s", hipGetErrorString(e));
    }
    for (auto &x : ev) (void)hipEventDestroy(x);
    if (result) return result;
    const hipMemcpyKind k = h->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPCHK(hipMemcpyAsync(x_out, snap.x, h->n * 8, k, h->stream));
    if (y_out && h->ny) HIPCHK(hipMemcpyAsync(y_out, snap.y, h->ny * 8, k, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    fill_info(h, snap, info, now_s() - t0, pass_secs, timed);
    return slot_status_code(snap.status);
}

// ---------------------------------------------------------------------------------------
// evaluations at an arbitrary point: anchor pass (FP64 accumulation) into the eval buffers

// anchor pass and epilogue at the point already in d_xe / d_ye -> d_ueval, d_geval
static qcqp_status eval_loaded_point(qcqp_handle *h)
{
    Slot S = h->hslot;
    reset_run_scalars(S);
    S.x = h->d_xe;
    S.y = h->d_ye;
    S.Uc[0] = h->d_ueval;
    S.Gc[0] = h->d_geval;
    HIPCHK(launch_fill(h->stream, h->d_ueval, (h->m + 1) * h->n, 0.0));   // rows of matrices not stored
    HIPCHK(hipMemcpyAsync(h->dslot_eval, &S, sizeof(Slot), hipMemcpyHostToDevice, h->stream));
    HIPCHK(launch_pass_only(h->stream, h->dslot_eval, h->dtiles, (int)h->tiles.size(), h->dstarts, h->B, h->dtype, (int)h->nw, h->pass_grid, h->nt,
                            h->sym64(), h->sym16()));
    HIPCHK(launch_epi_anchor(h->stream, h->dslot_eval, nullptr, 1, (int)(h->m + 1 + h->p)));
    return QCQP_OK;
}

static qcqp_status load_point(qcqp_handle *h, const double *x, const double *y, bool device_ptrs)
{
    const hipMemcpyKind k = device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (x != h->d_xe) HIPCHK(hipMemcpyAsync(h->d_xe, x, h->n * 8, k, h->stream));
    if (h->ny) {
        if (!y) HIPCHK(launch_fill(h->stream, h->d_ye, h->ny, 0.0));
        else if (y != h->d_ye) HIPCHK(hipMemcpyAsync(h->d_ye, y, h->ny * 8, k, h->stream));
    }
    return QCQP_OK;
}

static qcqp_status eval_point(qcqp_handle *h, const double *x, const double *y)
{
    if (h->owner) return fail(QCQP_E_INVALID, "handle is admitted to a batch");
    qcqp_status st = load_point(h, x, y, h->on_device != 0);
    if (st) return st;
    return eval_loaded_point(h);
}

// the handle's own G_xi scratch, (re)allocated when the handle first needs it
static qcqp_status ensure_gap_mem(qcqp_handle *h)
{
    const size_t need = (size_t)gap_scratch_doubles(h->n) * sizeof(double);
    if (h->gap_bytes < need) {
        if (h->gap_mem) (void)hipFree(h->gap_mem);
        h->gap_mem = nullptr;
        h->gap_bytes = 0;
        if (hipMalloc(&h->gap_mem, need) != hipSuccess) return fail(QCQP_E_NOMEM, "G_xi scratch (%zu bytes)", need);
        h->gap_bytes = need;
    }
    return QCQP_OK;
}

// G_xi at the device point (x_dev, y_dev) with `mem` (gap_scratch_doubles(n) doubles of device
// memory) as scratch, enqueued on h->stream with no host synchronisation: anchor pass and
// epilogue at the point, gradient, Py, H = Q(lambda) + 2 xi I, the box QP to convergence in one
// cooperative launch, Px.  *ctl_out receives the control words (ctl[9] = Py, ctl[10] = Px,
// ctl[4] = inner iterations).  Allocates nothing.
static qcqp_status gap_enqueue(qcqp_handle *h, const double *x_dev, const double *y_dev, double xi,
                               double *mem, double **ctl_out)
{
    qcqp_status st = load_point(h, x_dev, y_dev, true);
    if (st) return st;
    if ((st = eval_loaded_point(h))) return st;
    HIPCHK(launch_grad(h->stream, h->dslot_eval, (int)h->n, h->d_ueval, h->d_ye, h->d_grad));
    const int64_t n = h->n, ldh = round_up(n, 16);
    double *H = mem;
    double *v0 = H + n * ldh;
    const int64_t vs = round_up(n, 32);
    double *rowabs = v0, *Z = v0 + vs, *D = v0 + 2 * vs, *Dn = v0 + 3 * vs, *Hz = v0 + 4 * vs;
    double *part = v0 + 6 * vs, *ctl = part + 2 * GAP_MAX_BLOCKS;
    GridBar *bar = reinterpret_cast<GridBar *>(ctl + 32);
    // Z and D, then the barrier words (all-zero bits), cleared by a fill kernel rather than
    // memset nodes, so that a caller may capture this work into a graph
    static_assert(sizeof(GridBar) % sizeof(double) == 0, "GridBar is cleared as doubles");
    HIPCHK(launch_fill(h->stream, Z, 2 * vs, 0.0));
    HIPCHK(launch_fill(h->stream, reinterpret_cast<double *>(bar), sizeof(GridBar) / sizeof(double), 0.0));
    HIPCHK(launch_gap_setup(h->stream, h->dslot_eval, (int)n, (int)h->ny, h->d_ye, h->d_geval, h->d_grad, xi, H,
                            (int)ldh, rowabs, h->opt.inner_tol, ctl));
    // the LDS form uses Hz (written only after the loop) as the second step buffer
    HIPCHK(launch_fista_coop(h->stream, h->dslot_eval, (int)n, h->d_xe, h->d_grad, H, (int)ldh, Z, D, Dn, part, ctl,
                             h->opt.max_inner, bar, std::max(1, num_cus), max_lds, (int)(Hz - Dn)));
    HIPCHK(launch_gap_finish(h->stream, (int)n, h->d_grad, H, (int)ldh, (int)round_up(n, 2), D, Hz, ctl));
    *ctl_out = ctl;
    return QCQP_OK;
}

// G_xi at the device point, read back: out4 = {G, Py, Px, inner iterations}
static qcqp_status gap_at_device_point(qcqp_handle *h, const double *x_dev, const double *y_dev,
                                       double xi, double *mem, double *out4)
{
    double *ctl = nullptr;
    qcqp_status st = gap_enqueue(h, x_dev, y_dev, xi, mem, &ctl);
    if (st) return st;
    HIPCHK(hipMemcpyAsync(h->h_out, ctl, 11 * 8, hipMemcpyDeviceToHost, h->stream));
    unsigned berr = 0;
    HIPCHK(hipMemcpyAsync(&berr, &reinterpret_cast<GridBar *>(ctl + 32)->err, sizeof(unsigned),
                          hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (berr) return fail(QCQP_E_DEVICE, "G_xi inner loop: a grid barrier wait exceeded its limit");
    const double Py = h->h_out[9], Px = h->h_out[10];
    out4[0] = Py + Px;
    out4[1] = Py;
    out4[2] = Px;
    out4[3] = h->h_out[4];
    return QCQP_OK;
}

qcqp_status qcqp_eval_operator(qcqp_handle *h, const double *x, const double *y, double *Qx,
                               double *g, double *f, double *grad_x)
{
    g_err.clear();
    if (!h || !x) return fail(QCQP_E_INVALID, "null argument");
    if (h->owner) return fail(QCQP_E_INVALID, "handle is admitted to a batch");
    HIPCHK(join_streams(h->stream, h->ustream, h->ev_join));
    qcqp_status st;
    if ((st = eval_point(h, x, y))) return st;
    if (grad_x) HIPCHK(launch_grad(h->stream, h->dslot_eval, (int)h->n, h->d_ueval, h->d_ye, h->d_grad));
    const hipMemcpyKind k = h->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (Qx) HIPCHK(hipMemcpyAsync(Qx, h->d_ueval, (h->m + 1) * h->n * 8, k, h->stream));
    if (g && h->m) HIPCHK(hipMemcpyAsync(g, h->d_geval + h->p, h->m * 8, k, h->stream));
    if (f) HIPCHK(hipMemcpyAsync(f, h->d_geval + h->ny, 8, k, h->stream));
    if (grad_x) HIPCHK(hipMemcpyAsync(grad_x, h->d_grad, h->n * 8, k, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return QCQP_OK;
}

qcqp_status qcqp_eval_trial_pass(qcqp_handle *h, const double *x, const double *xc, int64_t nb,
                                 double *out)
{
    g_err.clear();
    if (!h || !x || !xc || !out) return fail(QCQP_E_INVALID, "null argument");
    if (h->owner) return fail(QCQP_E_INVALID, "handle is admitted to a batch");
    if (nb != h->B)
        return fail(QCQP_E_INVALID, "nb = %lld must equal options.spec_trials = %d", (long long)nb, h->B);
    HIPCHK(join_streams(h->stream, h->ustream, h->ev_join));
    Slot S = h->hslot;
    reset_run_scalars(S);
    S.mode = MODE_TRIAL;
    S.x = h->d_xe;
    const int64_t n = h->n, un = (h->m + 1) * n;
    const hipMemcpyKind kin = h->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const hipMemcpyKind kout = h->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPCHK(hipMemcpyAsync(S.x, x, n * 8, kin, h->stream));
    double *res[MAXB];
    for (int b = 0; b < h->B; ++b) {
        HIPCHK(hipMemcpyAsync(S.xc[b], xc + b * n, n * 8, kin, h->stream));
        res[b] = h->incremental ? S.W[b] : S.Uc[b];
        HIPCHK(hipMemsetAsync(res[b], 0, un * 8, h->stream));   // rows of matrices not stored
    }
    HIPCHK(hipMemcpyAsync(h->dslot_eval, &S, sizeof(Slot), hipMemcpyHostToDevice, h->stream));
    HIPCHK(launch_pass_only(h->stream, h->dslot_eval, h->dtiles, (int)h->tiles.size(), h->dstarts, h->B,
                            h->dtype, (int)h->nw, h->pass_grid, h->nt, h->sym64(), h->sym16()));
    for (int b = 0; b < h->B; ++b) HIPCHK(hipMemcpyAsync(out + b * un, res[b], un * 8, kout, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return QCQP_OK;
}

qcqp_status qcqp_eval_kkt(qcqp_handle *h, const double *x, const double *y, double *out6)
{
    g_err.clear();
    if (!h || !x || !out6) return fail(QCQP_E_INVALID, "null argument");
    if (h->owner) return fail(QCQP_E_INVALID, "handle is admitted to a batch");
    HIPCHK(join_streams(h->stream, h->ustream, h->ev_join));
    qcqp_status st;
    if ((st = eval_point(h, x, y))) return st;
    HIPCHK(launch_kkt(h->stream, h->dslot_eval, (int)h->n, (int)h->ny, h->d_xe, h->d_ye, h->d_ueval, h->d_geval,
                      h->d_kpart, h->d_out6));
    HIPCHK(hipMemcpyAsync(h->h_out, h->d_out6, 6 * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    std::memcpy(out6, h->h_out, 6 * 8);
    return QCQP_OK;
}

qcqp_status qcqp_eval_gap(qcqp_handle *h, const double *x, const double *y, double xi, double *out4)
{
    g_err.clear();
    if (!h || !x || !out4) return fail(QCQP_E_INVALID, "null argument");
    if (!(xi > 0.0)) return fail(QCQP_E_INVALID, "xi must be > 0");
    if (h->owner) return fail(QCQP_E_INVALID, "handle is admitted to a batch");
    HIPCHK(join_streams(h->stream, h->ustream, h->ev_join));
    qcqp_status st = load_point(h, x, y, h->on_device != 0);
    if (st) return st;
    if ((st = ensure_gap_mem(h))) return st;
    return gap_at_device_point(h, h->d_xe, h->d_ye, xi, h->gap_mem, out4);
}

qcqp_status qcqp_eval_gap_noalloc(qcqp_handle *h, const double *x, const double *y, double xi,
                                  double *out4)
{
    g_err.clear();
    if (!h || !x || !out4) return fail(QCQP_E_INVALID, "null argument");
    if (!(xi > 0.0)) return fail(QCQP_E_INVALID, "xi must be > 0");
    if (h->owner) return fail(QCQP_E_INVALID, "handle is admitted to a batch");
    if (h->n > QCQP_NOALLOC_MAX_N)
        return fail(QCQP_E_INVALID, "qcqp_eval_gap_noalloc: n = %lld exceeds QCQP_NOALLOC_MAX_N = %d",
                    (long long)h->n, QCQP_NOALLOC_MAX_N);
    double *mem = nullptr;
    qcqp_status st = static_scratch_for(h->dev, &mem);
    if (st) return st;
    HIPCHK(join_streams(h->stream, h->ustream, h->ev_join));
    if ((st = load_point(h, x, y, h->on_device != 0))) return st;
    return gap_at_device_point(h, h->d_xe, h->d_ye, xi, mem, out4);
}

// adaptive restart: evaluate G_xi at the slot's iterate (x_dev, y_dev from its last snapshot)
// and let the device decide on `decide_stream` (eq. (ada_restart)); nothing returns to the host
static qcqp_status run_gap_for(qcqp_handle *h, Slot *dslot, const double *x_dev, const double *y_dev,
                               hipStream_t decide_stream)
{
    qcqp_status st = ensure_gap_mem(h);
    if (st) return st;
    double *ctl = nullptr;
    if ((st = gap_enqueue(h, x_dev, y_dev, h->opt.xi, h->gap_mem, &ctl))) return st;
    if (decide_stream == h->stream) HIPCHK(launch_restart_decision_dev(h->stream, dslot, ctl));
    h->gap_ctl = ctl;
    return QCQP_OK;
}

qcqp_status qcqp_time_pass(qcqp_handle *h, int64_t reps, double *avg_seconds)
{
    g_err.clear();
    if (!h || !avg_seconds || reps < 1) return fail(QCQP_E_INVALID, "bad argument");
    if (h->owner) return fail(QCQP_E_INVALID, "handle is admitted to a batch");
    HIPCHK(join_streams(h->stream, h->ustream, h->ev_join));
    Slot S = h->hslot;
    reset_run_scalars(S);
    S.mode = MODE_TRIAL;
    HIPCHK(hipMemcpyAsync(h->dslot, &S, sizeof(Slot), hipMemcpyHostToDevice, h->stream));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(launch_pass_only(h->stream, h->dslot, h->dtiles, (int)h->tiles.size(), h->dstarts, h->B, h->dtype, (int)h->nw, h->pass_grid, h->nt,
                            h->sym64(), h->sym16()));
    HIPCHK(hipEventRecord(e0, h->stream));
    for (int64_t r = 0; r < reps; ++r)
        HIPCHK(launch_pass_only(h->stream, h->dslot, h->dtiles, (int)h->tiles.size(), h->dstarts, h->B, h->dtype, (int)h->nw, h->pass_grid, h->nt,
                            h->sym64(), h->sym16()));
    HIPCHK(hipEventRecord(e1, h->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_seconds = ms * 1e-3 / (double)reps;
    return QCQP_OK;
}

// ---------------------------------------------------------------------------------------
// continuous batching

qcqp_status qcqp_batch_create(const qcqp_options *opt, size_t budget, int64_t max_slots, qcqp_batch **out)
{
    g_err.clear();
    if (!out || max_slots < 1 || max_slots > 65535) return fail(QCQP_E_INVALID, "bad argument");
    qcqp_options o;
    if (opt) o = *opt;
    else qcqp_options_default(&o);
    qcqp_status st = validate_options(&o);
    if (st) return st;
    if ((st = ensure_prepared())) return st;
    qcqp_batch *bt = new (std::nothrow) qcqp_batch();
    if (!bt) return fail(QCQP_E_NOMEM, "host allocation");
    bt->opt = o;
    bt->budget = budget;
    bt->max_slots = max_slots;
    bt->ustream = (hipStream_t)o.stream;
    if (hipStreamCreateWithFlags(&bt->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&bt->gstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&bt->ev_join, hipEventDisableTiming) != hipSuccess) {
        if (bt->stream) (void)hipStreamDestroy(bt->stream);
        if (bt->gstream) (void)hipStreamDestroy(bt->gstream);
        delete bt;
        return fail(QCQP_E_DEVICE, "stream creation");
    }
    (void)hipGetDevice(&bt->dev);
    bt->gap_busy.assign(max_slots, 0);
    bt->gev.assign(max_slots, nullptr);
    bt->handles.assign(max_slots, nullptr);
    bt->finished.assign(max_slots, 0);
    bt->last_passes.assign(max_slots, 0);
    if (hipMalloc(&bt->dlive, max_slots * sizeof(int)) != hipSuccess ||
        hipMalloc(&bt->dslots, max_slots * sizeof(Slot)) != hipSuccess ||
        hipMalloc(&bt->ddesc, max_slots * sizeof(SymPass)) != hipSuccess ||
        hipHostMalloc((void **)&bt->h_poll, max_slots * sizeof(Slot)) != hipSuccess) {
        if (bt->dslots) (void)hipFree(bt->dslots);
        if (bt->dlive) (void)hipFree(bt->dlive);
        if (bt->ddesc) (void)hipFree(bt->ddesc);
        delete bt;
        return fail(QCQP_E_NOMEM, "slot table");
    }
    std::memset(bt->h_poll, 0, max_slots * sizeof(Slot));
    for (int64_t s = 0; s < max_slots; ++s) bt->h_poll[s].status = ST_IDLE;
    if (hipMemcpy(bt->dslots, bt->h_poll, max_slots * sizeof(Slot), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(bt->dslots);
        (void)hipFree(bt->dlive);
        (void)hipFree(bt->ddesc);
        (void)hipHostFree(bt->h_poll);
        delete bt;
        return fail(QCQP_E_DEVICE, "slot table init");
    }
    *out = bt;
    return QCQP_OK;
}

static size_t batch_resident(const qcqp_batch *bt)
{
    size_t s = 0;
    for (auto *h : bt->handles)
        if (h) s += h->q_bytes + h->arena_bytes + h->sym_bytes;
    return s;
}

qcqp_status qcqp_batch_stats(qcqp_batch *bt, int64_t *running, size_t *resident)
{
    if (!bt) return fail(QCQP_E_INVALID, "null batch");
    int64_t r = 0;
    for (int64_t s = 0; s < bt->max_slots; ++s)
        if (bt->handles[s] && !bt->finished[s]) ++r;
    if (running) *running = r;
    if (resident) *resident = batch_resident(bt);
    return QCQP_OK;
}

qcqp_status qcqp_batch_admit(qcqp_batch *bt, qcqp_handle *h, const double *x0, const double *y0, int64_t *slot)
{
    g_err.clear();
    if (!bt || !h || !slot) return fail(QCQP_E_INVALID, "null argument");
    if (h->owner) return fail(QCQP_E_INVALID, "handle already admitted");
    if (h->dtype != (int)bt->opt.storage || h->B != bt->opt.spec_trials || h->dev != bt->dev)
        return fail(QCQP_E_INVALID, "handle storage/spec_trials/device differ from the batch's");
    if (h->sym64()) return fail(QCQP_E_INVALID, "a handle created with sym_pass and F64 storage solves alone only");
    int64_t free_slot = -1;
    for (int64_t s = 0; s < bt->max_slots; ++s)
        if (!bt->handles[s]) { free_slot = s; break; }
    if (free_slot < 0) return fail(QCQP_E_NO_ROOM, "no free slot");
    if (bt->budget && batch_resident(bt) + h->q_bytes + h->arena_bytes + h->sym_bytes > bt->budget)
        return fail(QCQP_E_NO_ROOM, "HBM budget exhausted");
    // the handle's own stream work, and the caller's writes of x0 / y0, come first (stream
    // order only: the host does not wait)
    HIPCHK(join_streams(bt->stream, h->stream, h->ev_join));
    HIPCHK(join_streams(bt->stream, bt->ustream, bt->ev_join));
    hipStream_t saved = h->stream;
    h->stream = bt->stream;
    qcqp_status st = load_start(h, x0, y0);
    h->stream = saved;
    if (st) return st;
    Slot S = h->hslot;
    reset_run_scalars(S);
    bt->h_poll[free_slot] = S;
    HIPCHK(hipMemcpyAsync(bt->dslots + free_slot, &bt->h_poll[free_slot], sizeof(Slot),
                          hipMemcpyHostToDevice, bt->stream));
    HIPCHK(launch_start(bt->stream, bt->dslots + free_slot));
    if (h->sym16())
        HIPCHK(hipMemcpyAsync(bt->ddesc + free_slot, &h->sym, sizeof(SymPass), hipMemcpyHostToDevice, bt->stream));
    // The slot table entry is copied from pinned memory that only this slot's later polls
    // overwrite (queued behind the copy).  Caller-owned device start points are read by the
    // queued copies: wait for them before returning, so that the caller may reuse their memory.
    if (h->on_device && (x0 || y0)) HIPCHK(hipStreamSynchronize(bt->stream));
    bt->handles[free_slot] = h;
    bt->finished[free_slot] = 0;
    bt->last_passes[free_slot] = 0;
    h->owner = bt;
    bt->dirty = true;
    *slot = free_slot;
    return QCQP_OK;
}

static qcqp_status rebuild_tiles(qcqp_batch *bt)
{
    std::vector<Tile> all, all16;
    std::vector<int> live;
    std::vector<int2> work, work_r;
    size_t resident16 = 0;
    bt->max_nblk = 1;
    bt->max_ny = 1;
    bt->max_nw = 2;
    bt->max_epi = 1;
    bt->variants = 0;
    for (int64_t s = 0; s < bt->max_slots; ++s) {
        qcqp_handle *h = bt->handles[s];
        if (!h || bt->finished[s]) continue;
        live.push_back((int)s);
        // a packed slot's row-major tiles only serve its anchors: they go to their own launch,
        // so that they do not unbalance the trial-pass grid of the other slots
        std::vector<Tile> &dst = h->sym16() ? all16 : all;
        for (Tile t : h->tiles) {
            t.slot = (int32_t)s;
            dst.push_back(t);
        }
        if (h->sym16()) {
            for (int32_t t = 0; t < h->s16.nwork; ++t) work.push_back(int2{(int)s, t});
            for (int32_t k = 0; k < h->s16.nwork_r; ++k) work_r.push_back(int2{(int)s, k});
            resident16 += h->q_bytes;
        }

        bt->max_nblk = std::max(bt->max_nblk, h->nblk_step);
        bt->max_ny = std::max<int>(bt->max_ny, (int)h->ny);
        bt->max_nw = std::max<int>(bt->max_nw, (int)h->nw);
        bt->max_epi = std::max<int>(bt->max_epi, (int)(h->m + 1 + h->p));
        bt->variants |= h->hslot.variant == VAR_XY ? HAS_XY : HAS_YX;
    }
    // tiles stay grouped by slot: the pass grid gives each block a contiguous
    // range, so a block restages the iterate only at slot boundaries
    std::vector<Tile> &mixed = all;
    size_t resident = 0;
    for (int64_t s2 = 0; s2 < bt->max_slots; ++s2)
        if (bt->handles[s2] && !bt->finished[s2] && !bt->handles[s2]->sym16()) resident += bt->handles[s2]->q_bytes;
    bt->nt = (double)resident > CACHE_RESIDENT_BYTES ? 1 : 0;
    if (mixed.size() > bt->tiles_cap) {
        if (bt->dtiles) (void)hipFree(bt->dtiles);
        bt->dtiles = nullptr;
        size_t cap = std::max<size_t>(mixed.size() * 2, 1024);
        HIPCHK(hipMalloc(&bt->dtiles, cap * sizeof(Tile)));
        bt->tiles_cap = cap;
    }
    if (!mixed.empty())
        HIPCHK(hipMemcpyAsync(bt->dtiles, mixed.data(), mixed.size() * sizeof(Tile),
                              hipMemcpyHostToDevice, bt->stream));
    // byte-balanced ranges of the pass grid over the requests' tiles
    bt->pass_grid = pass_grid_for(bt->opt.spec_trials, (int)bt->opt.storage, bt->max_nw, (double)resident);
    {
        std::vector<int64_t> tb;
        tb.reserve(mixed.size());
        const int es = elem_size((int)bt->opt.storage);
        for (const Tile &t : mixed) tb.push_back((int64_t)t.nrows * bt->handles[t.slot]->n * es);
        const int grid = std::max(1, std::min<int>(bt->pass_grid, (int)mixed.size()));
        bt->starts_host = balanced_starts(tb, grid);
        if (bt->starts_host.size() > bt->starts_cap) {
            if (bt->dstarts) (void)hipFree(bt->dstarts);
            bt->dstarts = nullptr;
            const size_t cap = std::max<size_t>(bt->starts_host.size() * 2, 4096);
            HIPCHK(hipMalloc(&bt->dstarts, cap * sizeof(int)));
            bt->starts_cap = cap;
        }
        HIPCHK(hipMemcpyAsync(bt->dstarts, bt->starts_host.data(), bt->starts_host.size() * sizeof(int),
                              hipMemcpyHostToDevice, bt->stream));
    }
    if (!live.empty())
        HIPCHK(hipMemcpyAsync(bt->dlive, live.data(), live.size() * sizeof(int), hipMemcpyHostToDevice,
                              bt->stream));
    // the packed slots: anchor tiles with their own balanced grid, and the blocks of the tile and
    // row-sum kernels
    bt->has16 = !work.empty() || !all16.empty();
    if (bt->has16) {
        const int B = bt->opt.spec_trials, dt = (int)bt->opt.storage;
        if (all16.size() > bt->tiles16_cap) {
            if (bt->dtiles16) (void)hipFree(bt->dtiles16);
            bt->dtiles16 = nullptr;
            const size_t cap = std::max<size_t>(all16.size() * 2, 1024);
            HIPCHK(hipMalloc(&bt->dtiles16, cap * sizeof(Tile)));
            bt->tiles16_cap = cap;
        }
        if (!all16.empty())
            HIPCHK(hipMemcpyAsync(bt->dtiles16, all16.data(), all16.size() * sizeof(Tile), hipMemcpyHostToDevice,
                                  bt->stream));
        const int grid16 = std::max(1, std::min<int>(pass_grid_for(B, dt, bt->max_nw, (double)resident16),
                                                      (int)all16.size()));
        std::vector<int64_t> tb;
        for (const Tile &t : all16) tb.push_back((int64_t)t.nrows * bt->handles[t.slot]->n * elem_size(dt));
        bt->starts16_host = balanced_starts(tb, grid16);
        if (bt->starts16_host.size() > bt->starts16_cap) {
            if (bt->dstarts16) (void)hipFree(bt->dstarts16);
            bt->dstarts16 = nullptr;
            const size_t cap = std::max<size_t>(bt->starts16_host.size() * 2, 1024);
            HIPCHK(hipMalloc(&bt->dstarts16, cap * sizeof(int)));
            bt->starts16_cap = cap;
        }
        HIPCHK(hipMemcpyAsync(bt->dstarts16, bt->starts16_host.data(), bt->starts16_host.size() * sizeof(int),
                              hipMemcpyHostToDevice, bt->stream));
        bt->work_host = work;
        bt->work_host.insert(bt->work_host.end(), work_r.begin(), work_r.end());
        if (bt->work_host.size() > bt->work_cap) {
            if (bt->dwork) (void)hipFree(bt->dwork);
            bt->dwork = nullptr;
            const size_t cap = std::max<size_t>(bt->work_host.size() * 2, 4096);
            HIPCHK(hipMalloc(&bt->dwork, cap * sizeof(int2)));
            bt->work_cap = cap;
        }
        if (!bt->work_host.empty())
            HIPCHK(hipMemcpyAsync(bt->dwork, bt->work_host.data(), bt->work_host.size() * sizeof(int2),
                                  hipMemcpyHostToDevice, bt->stream));
        bt->s16 = Sym16Launch{dt, B, bt->ddesc, bt->dwork, (int32_t)work.size(), bt->dwork + work.size(),
                              (int32_t)work_r.size(), bt->dtiles16, (int32_t)all16.size(), grid16, bt->dstarts16};
    }
    bt->nlive = (int)live.size();
    bt->ntiles = (int)mixed.size();
    if (bt->gexec) (void)hipGraphExecDestroy(bt->gexec);   // launch shapes changed
    bt->gexec = nullptr;
    bt->dirty = false;
    return QCQP_OK;
}

qcqp_status qcqp_batch_step(qcqp_batch *bt, int64_t groups)
{
    g_err.clear();
    if (!bt || groups < 0) return fail(QCQP_E_INVALID, "bad argument");
    qcqp_status st;
    if (bt->dirty && (st = rebuild_tiles(bt))) return st;
    const bool timing = bt->opt.timing != 0;
    if (timing && (int64_t)bt->ev.size() < 2 * groups) {
        while ((int64_t)bt->ev.size() < 2 * groups) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            bt->ev.push_back(e);
        }
    }
    if (bt->nlive > 0) {
        auto launch_chunk = [&](hipStream_t s, bool with_events) -> hipError_t {
            for (int64_t g = 0; g < groups; ++g) {
                hipError_t e = launch_group(s, bt->dslots, bt->dlive, bt->nlive, bt->dtiles, bt->ntiles, bt->dstarts,
                                            bt->opt.spec_trials, (int)bt->opt.storage, bt->variants,
                                            bt->max_nblk,
                                            bt->max_ny, bt->max_nw, bt->max_epi, bt->pass_grid, bt->nt,
                                            with_events ? bt->ev[2 * g] : nullptr,
                                            with_events ? bt->ev[2 * g + 1] : nullptr, nullptr,
                                            bt->has16 ? &bt->s16 : nullptr);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        };
        hipError_t e;
        if (bt->opt.use_graphs && !timing) {
            if (!bt->gexec || bt->gexec_groups != groups) {
                if (bt->gexec) (void)hipGraphExecDestroy(bt->gexec);
                bt->gexec = nullptr;
                HIPCHK(capture_graph(bt->stream, [&](hipStream_t s) { return launch_chunk(s, false); }, &bt->gexec));
                bt->gexec_groups = groups;
            }
            e = hipGraphLaunch(bt->gexec, bt->stream);
        } else {
            e = launch_chunk(bt->stream, timing);
        }
        if (e != hipSuccess) return fail(QCQP_E_DEVICE, "launch: %s", hipGetErrorString(e));
    }
    HIPCHK(hipMemcpyAsync(bt->h_poll, bt->dslots, bt->max_slots * sizeof(Slot), hipMemcpyDeviceToHost, bt->stream));
    HIPCHK(hipStreamSynchronize(bt->stream));
    if (timing && bt->nlive > 0) {
        for (int64_t g = 0; g < groups; ++g) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, bt->ev[2 * g], bt->ev[2 * g + 1]) == hipSuccess) bt->pass_seconds += ms * 1e-3;
        }
    }
    for (int64_t s = 0; s < bt->max_slots; ++s) {
        qcqp_handle *h = bt->handles[s];
        if (!h) continue;
        const int64_t d = bt->h_poll[s].passes - bt->last_passes[s];
        if (d > 0) {
            const double nn = h->sym16() ? (double)h->n * (double)(h->n + 1) / 2 : (double)h->n * (double)h->n;
            bt->pass_bytes += (double)d * (double)h->nq * nn * elem_size(h->dtype);
            bt->passes += d;
        }
        bt->last_passes[s] = bt->h_poll[s].passes;
    }
    // adaptive restarts pending: each pending slot's G_xi runs on the batch's gap stream while
    // the other slots keep stepping; once it has completed, the decision (on the device, from
    // the device's G_xi) is enqueued on the batch stream ahead of the next groups
    for (int64_t s = 0; s < bt->max_slots; ++s) {
        qcqp_handle *h = bt->handles[s];
        if (!h || bt->finished[s]) continue;
        const Slot &S = bt->h_poll[s];
        if (S.status == ST_GAP_PENDING) {
            if (!bt->gap_busy[s]) {
                if (!bt->gev[s]) HIPCHK(hipEventCreateWithFlags(&bt->gev[s], hipEventDisableTiming));
                hipStream_t saved = h->stream;
                h->stream = bt->gstream;
                st = run_gap_for(h, bt->dslots + s, S.x, S.y, nullptr);
                h->stream = saved;
                if (st) return st;
                HIPCHK(hipEventRecord(bt->gev[s], bt->gstream));
                bt->gap_busy[s] = 1;
            } else {
                const hipError_t q = hipEventQuery(bt->gev[s]);
                if (q == hipSuccess) {
                    HIPCHK(launch_restart_decision_dev(bt->stream, bt->dslots + s, h->gap_ctl));
                    bt->gap_busy[s] = 0;
                } else if (q != hipErrorNotReady) {
                    return fail(QCQP_E_DEVICE, "G_xi of slot %lld: %s", (long long)s, hipGetErrorString(q));
                }
            }
        } else if (S.status != ST_RUNNING) {
            if (!bt->finished[s]) {
                bt->finished[s] = 1;
                bt->dirty = true;
            }
        }
    }
    return QCQP_OK;
}

qcqp_status qcqp_batch_pass_stats(qcqp_batch *bt, double *pass_seconds, double *pass_bytes, int64_t *passes)
{
    if (!bt) return fail(QCQP_E_INVALID, "null batch");
    if (pass_seconds) *pass_seconds = bt->pass_seconds;
    if (pass_bytes) *pass_bytes = bt->pass_bytes;
    if (passes) *passes = bt->passes;
    return QCQP_OK;
}

qcqp_status qcqp_batch_poll(qcqp_batch *bt, int64_t *done, int64_t cap, int64_t *n_done)
{
    if (!bt || !n_done) return fail(QCQP_E_INVALID, "bad argument");
    int64_t c = 0;
    for (int64_t s = 0; s < bt->max_slots; ++s)
        if (bt->handles[s] && bt->finished[s]) {
            if (done && c < cap) done[c] = s;
            ++c;
        }
    *n_done = std::min(c, cap);
    return QCQP_OK;
}

qcqp_status qcqp_batch_fetch(qcqp_batch *bt, int64_t slot, double *x_out, double *y_out,
                             qcqp_info *info, qcqp_handle **h_out)
{
    g_err.clear();
    if (!bt || slot < 0 || slot >= bt->max_slots || !bt->handles[slot])
        return fail(QCQP_E_INVALID, "no such slot");
    if (!bt->finished[slot]) return fail(QCQP_E_INVALID, "slot %lld is still running", (long long)slot);
    qcqp_handle *h = bt->handles[slot];
    const Slot S = bt->h_poll[slot];   // a copy: the table entry is marked idle below
    const hipMemcpyKind k = h->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (x_out) HIPCHK(hipMemcpyAsync(x_out, S.x, h->n * 8, k, bt->stream));
    if (y_out && h->ny) HIPCHK(hipMemcpyAsync(y_out, S.y, h->ny * 8, k, bt->stream));
    // mark the device slot idle so later groups skip it
    Slot idle = S;
    idle.status = ST_IDLE;
    bt->h_poll[slot] = idle;
    HIPCHK(hipMemcpyAsync(bt->dslots + slot, &bt->h_poll[slot], sizeof(Slot), hipMemcpyHostToDevice, bt->stream));
    HIPCHK(hipStreamSynchronize(bt->stream));
    fill_info(h, S, info, 0.0, 0.0, 0);
    if (info) {
        switch (S.status) {
        case ST_CONVERGED: info->status = QCQP_OK; break;
        case ST_MAX_ITER: info->status = QCQP_E_NOT_CONVERGED; break;
        default: info->status = QCQP_E_NUMERICAL; break;
        }
    }
    bt->handles[slot] = nullptr;
    bt->finished[slot] = 0;
    h->owner = nullptr;
    if (h_out) *h_out = h;
    bt->dirty = true;
    return QCQP_OK;
}

qcqp_status qcqp_batch_destroy(qcqp_batch *bt)
{
    if (!bt) return QCQP_OK;
    (void)hipStreamSynchronize(bt->stream);
    (void)hipStreamSynchronize(bt->gstream);
    for (auto *h : bt->handles)
        if (h) {
            h->owner = nullptr;
            free_handle_memory(h);
            delete h;
        }
    if (bt->dslots) (void)hipFree(bt->dslots);
    if (bt->h_poll) (void)hipHostFree(bt->h_poll);
    if (bt->dtiles) (void)hipFree(bt->dtiles);
    if (bt->dstarts) (void)hipFree(bt->dstarts);
    if (bt->dlive) (void)hipFree(bt->dlive);
    if (bt->ddesc) (void)hipFree(bt->ddesc);
    if (bt->dtiles16) (void)hipFree(bt->dtiles16);
    if (bt->dstarts16) (void)hipFree(bt->dstarts16);
    if (bt->dwork) (void)hipFree(bt->dwork);
    for (auto &e : bt->ev) (void)hipEventDestroy(e);
    if (bt->gexec) (void)hipGraphExecDestroy(bt->gexec);
    if (bt->ev_join) (void)hipEventDestroy(bt->ev_join);
    for (auto &e : bt->gev)
        if (e) (void)hipEventDestroy(e);
    if (bt->stream) (void)hipStreamDestroy(bt->stream);
    if (bt->gstream) (void)hipStreamDestroy(bt->gstream);
    delete bt;
    return QCQP_OK;
}

}  // extern "C"

