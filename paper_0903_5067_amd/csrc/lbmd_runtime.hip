// Host runtime and C ABI of the fluctuating D3Q19 LB library (include/lbmd.h).
//
// Lays out the caller-owned device buffers, validates the box descriptions,
// prepares the per-box constants the kernels read, orders the launches of one
// LB step (couple -> collide -> fixup, Sec. II.B: the coupling hands the
// beads' momentum to the fluid, then the LB equation collides and streams),
// records them into HIP graphs on request, and moves observables and state
// across the host boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbmd.h"
#include "lbmd_kernels.hpp"

using namespace lbd;

// Device memory of lb_observables_static: the partial sums of its reduction
// live in this file-scope array instead of the caller's scratch buffer, for
// callers that cannot allocate.  Each device the library runs on holds its
// own copy, at its own address, until the process ends.  In host code the
// name stands for a host-side symbol, not a device address: kernels receive
// the address hipGetSymbolAddress gives for the current device (static_scratch).
constexpr size_t STATIC_SCRATCH_BYTES = LB_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[MAX_DEVICES] = {};

// the device address of `scratch` on device dev (the current device), looked
// up once per device; null if the runtime could not give it
void* static_scratch(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_dev[dev] = p;
        else (void)hipGetLastError();
    }
    return g_scratch_dev[dev];
}

thread_local std::string g_err;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
uint64_t round_up(uint64_t x, uint64_t m) { return (x + m - 1) / m * m; }

constexpr int NL_CAP = NL_SLOTS;   // neighbour-list entries per bead
constexpr double MODE_B[19] = {1, 1. / 3, 1. / 3, 1. / 3, 2. / 3, 4. / 3, 4. / 9, 1. / 9, 1. / 9, 1. / 9,
                               2. / 3, 2. / 3, 2. / 3, 2. / 9, 2. / 9, 2. / 9, 2, 4. / 3, 4. / 9};

struct Layout {
    size_t esz = 8;
    std::vector<uint64_t> pop_off, bead_off, V, node_off;
    std::vector<uint32_t> tile_begin, n_tiles;
    std::vector<uint8_t> dense;                       // per box: collide after the coupling, no fix-up
    std::vector<uint64_t> field_off;                  // per box: first node in the velocity field (dense boxes)
    uint64_t field_nodes = 0;                         // nodes of all dense boxes
    std::vector<uint64_t> bin_off, item_off;          // per box: its run bins and binned runs (dense boxes)
    uint64_t bin_entries = 0, item_entries = 0;
    uint32_t dense_max_tiles = 0;                     // collide tiles of the largest dense box
    uint64_t tiles_sparse = 0, beads_sparse = 0;      // collide tiles (first in tile order) and beads of the other boxes
    uint64_t pop_elems = 0, total_tiles = 0, total_beads = 0, total_nodes = 0;
    std::vector<uint32_t> stat_off;                   // per box: first observable partial record
    uint32_t stat_recs = 0, stat_max_recs = 0;        // records of all boxes, of the largest box
    size_t st_popA = 0, st_popB = 0, st_x = 0, st_v = 0, st_f = 0, st_fc = 0, state_bytes = 0;
    size_t sc_ctrl = 0, sc_boxes = 0, sc_ccs = 0, sc_tilebox = 0, sc_couple = 0, sc_imp = 0, sc_claim = 0,
           sc_touched = 0, sc_tcnt = 0, sc_beadbox = 0, sc_nlcnt = 0, sc_nlidx = 0, sc_nlx0 = 0,
           sc_part = 0, sc_mid = 0, sc_stat = 0, sc_chain = 0, sc_vhist = 0, sc_nlreb = 0, sc_biglist = 0, sc_alllist = 0,
           sc_nearu = 0, sc_nearc = 0, sc_subrec = 0, sc_field = 0, sc_binstart = 0, sc_items = 0, sc_slotof = 0,
           sc_defer = 0, sc_dclaim = 0, sc_dlist = 0, sc_ovf = 0, sc_ovm = 0, scratch_bytes = 0;
    uint64_t beads_big_sparse = 0;                    // beads of the chains above BIG_CHAIN in the other boxes
    uint32_t defer_cap = 0, ovf_cap = 0;              // deferred-tile list and overflow list entries
    int max_N = 0;         // largest chain taking the one-workgroup path
    std::vector<int32_t> big_list;                    // boxes whose chain takes the 1024-thread kernel
    int big_max_n = 0, big_max_sub = 0;              // largest chain and most substeps among them
    std::vector<int32_t> small_list;                  // boxes on the one-workgroup path
    std::vector<int> couple_T;   // per box: lanes per bead on the one-workgroup path
    int couple_block = 64;
    int touch_cap = 8;
};

bool validate(const lb_box_desc* b, int32_t n, int32_t prec, int32_t hist, std::string& err)
{
    if (!b || n <= 0) { err = "need at least one box"; return false; }
    if (prec != LB_FP64 && prec != LB_FP32_DEV) { err = "precision must be LB_FP64 or LB_FP32_DEV"; return false; }
    if (hist < 0) { err = "hist_steps must be >= 0"; return false; }
    for (int i = 0; i < n; ++i) {
        const lb_box_desc& d = b[i];
        auto bad = [&](const char* what) { err = "box " + std::to_string(i) + ": " + what; return false; };
        if (d.L < 2 || d.L > 1625) return bad("L must be in [2, 1625]");
        const uint64_t V = (uint64_t)d.L * d.L * d.L;
        if (d.n_beads < 0 || d.n_beads > 1024 || (uint64_t)d.n_beads > V) return bad("N must be in [0, min(1024, L^3)]");
        if (d.chain_len < 0 || (d.chain_len > 0 && d.n_beads > 0 && d.n_beads % d.chain_len != 0))
            return bad("chain_len must be 0 or divide N");
        if (!(d.rho0 > 0)) return bad("rho0 must be > 0");
        for (double w : {d.omega_shear, d.omega_bulk, d.omega_ghost})
            if (!(w > 0 && w < 2)) return bad("relaxation rates must be in (0, 2)");
        if (!(d.kT >= 0)) return bad("kT must be >= 0");
        if (d.thermalize < 0 || d.thermalize > 2) return bad("thermalize must be 0, 1 or 2");
        if (!(d.md_dt > 0) || d.md_substeps < 1) return bad("md_dt > 0 and md_substeps >= 1 required");
        if (!(std::fabs(d.md_substeps * d.md_dt - d.tau_lb) <= 1e-12 * d.tau_lb) || !(d.tau_lb > 0))
            return bad("tau_lb must equal md_substeps * md_dt");
        if (!(d.bead_mass > 0) || !(d.zeta >= 0) || !(d.k_fene >= 0) || !(d.r0_fene > 0) ||
            !(d.eps_wca >= 0) || !(d.sigma_wca > 0))
            return bad("chain parameters out of range");
    }
    return true;
}

Layout make_layout(const lb_box_desc* b, int32_t n, int32_t prec, int32_t hist)
{
    Layout Lo;
    Lo.esz = prec == LB_FP64 ? 8 : 4;
    uint64_t pop = 0, tiles = 0, beads = 0, nodes = 0;
    int max_sub = 1;
    for (int i = 0; i < n; ++i) max_sub = std::max(max_sub, b[i].md_substeps);
    Lo.touch_cap = 8 * (max_sub + 1);
    for (int i = 0; i < n; ++i) {
        const uint64_t V = (uint64_t)b[i].L * b[i].L * b[i].L;
        Lo.V.push_back(V);
        Lo.pop_off.push_back(pop);
        pop += pop_elems_of(V);   // whole tiles of PTILE nodes (4 or 8 KB per plane)
        Lo.n_tiles.push_back((uint32_t)((V + 255) / 256));
        tiles += (V + 255) / 256;
        Lo.stat_off.push_back(Lo.stat_recs);
        Lo.stat_recs += stat_recs_of(Lo.n_tiles.back());
        Lo.stat_max_recs = std::max(Lo.stat_max_recs, stat_recs_of(Lo.n_tiles.back()));
        // a chain on the workgroup path whose stencils (8 nodes per bead)
        // cover a quarter of the box or more: re-colliding its nodes in a
        // fix-up would cost more than colliding the box after the coupling
        Lo.dense.push_back(b[i].n_beads > BIG_CHAIN && 32 * (uint64_t)b[i].n_beads >= V ? 1 : 0);
        Lo.field_off.push_back(Lo.field_nodes);
        Lo.bin_off.push_back(Lo.bin_entries);
        Lo.item_off.push_back(Lo.item_entries);
        if (Lo.dense.back()) {
            Lo.field_nodes += V;
            Lo.bin_entries += V + 1;
            Lo.item_entries += (uint64_t)b[i].n_beads * (uint64_t)b[i].md_substeps;
            Lo.dense_max_tiles = std::max(Lo.dense_max_tiles, (uint32_t)((V + 255) / 256));
        } else {
            Lo.beads_sparse += (uint64_t)b[i].n_beads;
        }
        Lo.bead_off.push_back(beads);
        beads += b[i].n_beads;
        Lo.node_off.push_back(nodes);
        nodes += V;
        const int N = b[i].n_beads;
        if (N > BIG_CHAIN) {
            if (!Lo.dense.back()) Lo.beads_big_sparse += (uint64_t)N;
            Lo.big_list.push_back(i);
            Lo.big_max_n = std::max(Lo.big_max_n, N);
            Lo.big_max_sub = std::max(Lo.big_max_sub, b[i].md_substeps);
        } else if (N > 0) {
            Lo.small_list.push_back(i);
            Lo.max_N = std::max(Lo.max_N, N);
        }
    }
    // collide tiles: the other boxes first, dense boxes after them, so that
    // each group is one contiguous range
    uint64_t t0 = 0;
    Lo.tile_begin.assign(n, 0);
    for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < n; ++i)
            if (Lo.dense[i] == pass) {
                Lo.tile_begin[i] = (uint32_t)t0;
                t0 += Lo.n_tiles[i];
                if (pass == 0) Lo.tiles_sparse = t0;
            }
    Lo.pop_elems = pop;
    Lo.total_tiles = tiles;
    Lo.total_beads = beads;
    Lo.total_nodes = nodes;
    // lanes per bead in the coupling workgroup: split the pair loop while the
    // chain is small (a function of the box's own N, so that a box computes
    // the same bits alone and in any batch), one lane per bead otherwise
    int widest = 0;
    for (int i = 0; i < n; ++i) {
        const int N = b[i].n_beads;
        int T = 1;
        if (N > 0 && N <= BIG_CHAIN)
            while (T < 16 && 2 * T * N <= 256) T *= 2;
        Lo.couple_T.push_back(T);
        if (N > 0 && N <= BIG_CHAIN) widest = std::max(widest, T * N);
    }
    if (widest > 0) Lo.couple_block = (int)round_up((uint64_t)widest, 64);
    size_t o = 0;
    Lo.st_popA = o; o = align256(o + pop * Lo.esz);
    Lo.st_popB = o; o = align256(o + pop * Lo.esz);
    const size_t bb = std::max<uint64_t>(beads, 1) * 3 * sizeof(double);
    Lo.st_x = o; o = align256(o + bb);
    Lo.st_v = o; o = align256(o + bb);
    Lo.st_f = o; o = align256(o + bb);
    Lo.st_fc = o; o = align256(o + bb);
    Lo.state_bytes = o;
    o = 0;
    const size_t ccsz = prec == LB_FP64 ? sizeof(CollideConst<double>) : sizeof(CollideConst<float>);
    Lo.sc_ctrl = o; o = align256(o + sizeof(Ctrl));
    Lo.sc_boxes = o; o = align256(o + n * sizeof(BoxDev));
    Lo.sc_ccs = o; o = align256(o + n * ccsz);
    Lo.sc_tilebox = o; o = align256(o + tiles * sizeof(uint32_t));
    Lo.sc_couple = o; o = align256(o + n * sizeof(int32_t));
    const uint64_t impn = beads ? nodes : 1;   // the impulse field exists only when there are beads
    Lo.sc_imp = o; o = align256(o + impn * 3 * sizeof(unsigned long long));
    Lo.sc_claim = o; o = align256(o + impn * sizeof(uint32_t));
    const uint64_t nbx = std::max<uint64_t>(beads, 1);
    Lo.sc_touched = o; o = align256(o + nbx * Lo.touch_cap * sizeof(uint32_t));
    Lo.sc_tcnt = o; o = align256(o + nbx * sizeof(int32_t));
    Lo.sc_beadbox = o; o = align256(o + nbx * sizeof(int32_t));
    Lo.sc_nlcnt = o; o = align256(o + nbx * sizeof(int32_t));
    Lo.sc_nlidx = o; o = align256(o + nbx * NL_CAP * sizeof(uint16_t));
    Lo.sc_nlx0 = o; o = align256(o + std::max<uint64_t>(beads, 1) * 3 * sizeof(double));
    Lo.sc_part = o; o = align256(o + (size_t)Lo.stat_recs * NSTAT_REC * sizeof(double));
    Lo.sc_mid = o; o = align256(o + (size_t)n * STAT_CHUNKS * NSTAT_REC * sizeof(double));
    Lo.sc_stat = o; o = align256(o + n * NSTAT_REC * sizeof(double));
    Lo.sc_chain = o; o = align256(o + n * NCHAIN_REC * sizeof(double));
    Lo.sc_vhist = o; o = align256(o + (size_t)hist * std::max<uint64_t>(beads, 1) * 3 * sizeof(double));
    Lo.sc_nlreb = o; o = align256(o + n * sizeof(uint32_t));
    Lo.sc_biglist = o; o = align256(o + n * sizeof(int32_t));
    Lo.sc_alllist = o; o = align256(o + n * sizeof(int32_t));
    {   // tables of the large-chain kernels, sized only when there are such chains
        const uint64_t nbig = Lo.big_list.empty() ? 1 : nbx;
        Lo.sc_nearu = o; o = align256(o + nbig * 27 * 3 * Lo.esz);
        Lo.sc_nearc = o; o = align256(o + nbig * 4 * sizeof(int32_t));
        Lo.sc_subrec = o; o = align256(o + (uint64_t)std::max(Lo.big_max_sub, 1) * nbig * 8 * sizeof(double));
        Lo.sc_field = o; o = align256(o + std::max<uint64_t>(Lo.field_nodes, 1) * 3 * Lo.esz);
        Lo.sc_binstart = o; o = align256(o + std::max<uint64_t>(Lo.bin_entries, 1) * sizeof(uint32_t));
        Lo.sc_items = o; o = align256(o + std::max<uint64_t>(Lo.item_entries, 1) * 24 * sizeof(unsigned long long));
        Lo.sc_slotof = o; o = align256(o + std::max<uint64_t>(Lo.item_entries, 1) * sizeof(uint32_t));
        // deferred segments (64 nodes, four per collide tile): three step
        // stamps per segment (deferred in the steps of either parity, listed
        // in); a segment is listed once, and a bead's table spans at most
        // 27.  A bead hands impulses to at most 8 new nodes per substep.
        Lo.defer_cap = (uint32_t)(27 * Lo.beads_big_sparse);
        Lo.ovf_cap = (uint32_t)(8 * (uint64_t)std::max(Lo.big_max_sub, 1) * Lo.beads_big_sparse);
        Lo.sc_defer = o; o = align256(o + (Lo.beads_big_sparse ? 2 * DSEG_PER_TILE * tiles : 1) * sizeof(uint32_t));
        Lo.sc_dclaim = o; o = align256(o + (Lo.beads_big_sparse ? DSEG_PER_TILE * tiles : 1) * sizeof(uint32_t));
        Lo.sc_dlist = o; o = align256(o + std::max<uint32_t>(Lo.defer_cap, 1) * sizeof(uint32_t));
        Lo.sc_ovf = o; o = align256(o + std::max<uint32_t>(Lo.ovf_cap, 1) * 2 * sizeof(uint32_t));
        Lo.sc_ovm = o; o = align256(o + (Lo.beads_big_sparse ? nodes : 1) * sizeof(uint32_t));
    }
    Lo.scratch_bytes = o;
    return Lo;
}

template <typename R>
CollideConst<R> collide_const(const lb_box_desc& d)
{
    CollideConst<R> c;
    const double gb = 1 - d.omega_bulk, gs = 1 - d.omega_shear, gg = 1 - d.omega_ghost;
    c.rho0 = (R)d.rho0;
    c.gb = (R)gb; c.gs = (R)gs; c.gg = (R)gg;
    c.hb = (R)(0.5 * (1 + gb)); c.hs = (R)(0.5 * (1 + gs));
    // mu = kT_lat / c_s^2, kT_lat = kT tau_lb^2 (lattice spacing and mass unit 1)
    c.mu = (R)(3.0 * d.kT * d.tau_lb * d.tau_lb);
    c.therm = d.thermalize;
    for (int k = 0; k < 19; ++k) {
        const double g = k == 4 ? gb : (k < 10 ? gs : gg);
        c.q[k] = k < 4 ? (R)0 : (R)std::sqrt((1 - g * g) / MODE_B[k]);
    }
    return c;
}

}  // namespace

struct lb_handle {
    int n_boxes = 0;
    int dev = 0;                      // the device the handle was set up on
    void* static_scr = nullptr;       // that device's address of the static array (lb_observables_static)
    int prec = LB_FP32_DEV;
    int hist = 0;
    std::vector<lb_box_desc> desc;
    Layout lo;
    char* state = nullptr;
    char* scratch = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // the chain coupling runs on a second stream, concurrently with the
    // collide kernel of the same step (both only read the current state)
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_table = nullptr, ev_head = nullptr, ev_def = nullptr;
    hipEvent_t ev_coll = nullptr;     // chain-bound runs: this step's collide is done
    LaunchCtx ctx{};
    LaunchCtx ctx2{};
    int32_t* couple_list = nullptr;   // device: boxes on the one-workgroup path (chains <= 256 beads)
    int32_t* big_list = nullptr;      // device: boxes with chains of 257..1024 beads
    std::vector<int32_t> couple_host; // box indices with beads
    std::vector<BoxDev> boxes_host;   // host copy of the device box table
    int cur = 0;                      // 0: buffer A holds the current state
    uint64_t step = 0;                // host mirror of the device step counter
    bool pending = false;             // lb_couple done, impulses not yet consumed
    int batched = 1;
    int overlap = 1;                  // batched steps defer the tiles around large chains (see enqueue_step)
    int resident = 1;                 // runs may keep a chain kernel waiting for a later collide (fused_steps)
    int graph_steps = 0;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    std::string err;
    // adjoint window
    int win_T = 0, win_k = 0;
    uint64_t win_step0 = 0;
    bool win_ready = false;        // a forward window is recorded in the workspace
    void* ccd = nullptr;           // device CollideConst<double>[n_boxes] for the reverse sweep

    void* pop(int which) { return state + (which == 0 ? lo.st_popA : lo.st_popB); }
};

namespace {

lb_status fail(lb_handle* h, lb_status s, const std::string& msg)
{
    if (h) h->err = msg; else g_err = msg;
    return s;
}

#define HIPCHK(h, call)                                                                         \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(h, LB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

// zero every per-node and per-tile step stamp and the step-tagged control
// words (after the step count is set back), on the handle's stream, then
// wait for it; outside any graph
hipError_t clear_step_stamps(lb_handle* h, bool sync = true)
{
    const Layout& lo = h->lo;
    if (!lo.total_beads) return hipSuccess;
    char* ctrl = h->scratch + lo.sc_ctrl;
    hipError_t e = hipMemsetAsync(h->scratch + lo.sc_claim, 0, lo.total_nodes * sizeof(uint32_t), h->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(ctrl + offsetof(Ctrl, ovf_flag), 0, sizeof(Ctrl) - offsetof(Ctrl, ovf_flag), h->stream);
    if (e == hipSuccess && lo.beads_big_sparse) {
        e = hipMemsetAsync(h->scratch + lo.sc_defer, 0, 2 * DSEG_PER_TILE * lo.total_tiles * sizeof(uint32_t),
                           h->stream);
        if (e == hipSuccess)
            e = hipMemsetAsync(h->scratch + lo.sc_dclaim, 0, DSEG_PER_TILE * lo.total_tiles * sizeof(uint32_t),
                               h->stream);
        if (e == hipSuccess)
            e = hipMemsetAsync(h->scratch + lo.sc_ovm, 0, lo.total_nodes * sizeof(uint32_t), h->stream);
    }
    if (e == hipSuccess && sync) e = hipStreamSynchronize(h->stream);
    return e;
}

// one LB step's launches with relative step offset s_off, from buffer `from`
lb_status enqueue_step(lb_handle* h, int from, uint32_t s_off, bool couple)
{
    const void* A = h->pop(from);
    void* B = h->pop(1 - from);
    const bool f64 = h->prec == LB_FP64;
    const LaunchCtx& c = h->ctx;
    const int nc = (int)h->couple_host.size();
    const bool any_beads = h->lo.total_beads > 0;
    if (h->batched) {
        const bool fork = couple && any_beads;
        const int nbig = (int)h->lo.big_list.size();
        // chains above BIG_CHAIN beads in sparse boxes: the tiles around
        // them are collided beside the plain collide once their impulses are
        // in, instead of re-collided after it (same bits either way)
        const bool defer = fork && h->overlap && h->lo.beads_big_sparse > 0 && !c.keep_imp && !c.tape;
        LaunchCtx c1 = c;
        c1.defer_on = defer ? 1 : 0;
        if (fork) {
            HIPCHK(h, hipEventRecord(h->ev_fork, h->stream));
            HIPCHK(h, hipStreamWaitEvent(h->stream2, h->ev_fork, 0));
            LaunchCtx c2 = h->ctx2;
            c2.defer_on = c1.defer_on;
            // a chain above 256 beads needs a whole CU (1024 threads, the full
            // register file): the collide waits for its short node-table
            // kernel, so the chain kernel queued right behind it is dispatched
            // onto an idle GPU instead of behind the collide's workgroups
            if (nbig)
                HIPCHK(h, f64 ? launch_couple_big<double>(c2, A, h->big_list, nbig, h->lo.big_max_n, s_off, h->ev_table)
                              : launch_couple_big<float>(c2, A, h->big_list, nbig, h->lo.big_max_n, s_off, h->ev_table));
            if (nc)
                HIPCHK(h, f64 ? launch_couple<double>(c2, A, h->couple_list, nc, h->lo.couple_block, s_off)
                              : launch_couple<float>(c2, A, h->couple_list, nc, h->lo.couple_block, s_off));
            if (defer)
                HIPCHK(h, f64 ? launch_collide_deferred<double>(c2, A, B, s_off)
                              : launch_collide_deferred<float>(c2, A, B, s_off));
            HIPCHK(h, hipEventRecord(h->ev_join, h->stream2));
            if (nbig) HIPCHK(h, hipStreamWaitEvent(h->stream, h->ev_table, 0));
        }
        const uint32_t ts = (uint32_t)h->lo.tiles_sparse, td = (uint32_t)(h->lo.total_tiles - h->lo.tiles_sparse);
        HIPCHK(h, f64 ? launch_collide<double>(c1, A, B, -1, 0, ts, s_off)
                      : launch_collide<float>(c1, A, B, -1, 0, ts, s_off));
        if (fork) HIPCHK(h, hipStreamWaitEvent(h->stream, h->ev_join, 0));
        if (h->lo.beads_sparse > (defer ? h->lo.beads_big_sparse : 0))
            HIPCHK(h, f64 ? launch_fixup<double>(c1, A, B, 0, h->lo.total_beads, s_off)
                          : launch_fixup<float>(c1, A, B, 0, h->lo.total_beads, s_off));
        if (defer)
            HIPCHK(h, f64 ? launch_overflow<double>(c1, A, B, s_off) : launch_overflow<float>(c1, A, B, s_off));
        HIPCHK(h, f64 ? launch_collide_forced<double>(c, A, B, -1, ts, td, s_off)
                      : launch_collide_forced<float>(c, A, B, -1, ts, td, s_off));
    } else {
        for (int i = 0; i < nc; ++i) {
            if (!couple) break;
            HIPCHK(h, f64 ? launch_couple<double>(c, A, h->couple_list + i, 1, h->lo.couple_block, s_off)
                          : launch_couple<float>(c, A, h->couple_list + i, 1, h->lo.couple_block, s_off));
        }
        for (int k = 0; k < (int)h->lo.big_list.size() && couple; ++k) {
            const int nk = h->desc[h->lo.big_list[k]].n_beads;
            HIPCHK(h, f64 ? launch_couple_big<double>(c, A, h->big_list + k, 1, nk, s_off, nullptr)
                          : launch_couple_big<float>(c, A, h->big_list + k, 1, nk, s_off, nullptr));
        }
        for (int b = 0; b < h->n_boxes; ++b) {
            if (h->lo.dense[b]) {
                HIPCHK(h, f64 ? launch_collide_forced<double>(c, A, B, b, h->lo.tile_begin[b], h->lo.n_tiles[b], s_off)
                              : launch_collide_forced<float>(c, A, B, b, h->lo.tile_begin[b], h->lo.n_tiles[b], s_off));
                continue;
            }
            HIPCHK(h, f64 ? launch_collide<double>(c, A, B, b, h->lo.tile_begin[b], h->lo.n_tiles[b], s_off)
                          : launch_collide<float>(c, A, B, b, h->lo.tile_begin[b], h->lo.n_tiles[b], s_off));
            const uint64_t nb = (uint64_t)h->desc[b].n_beads;
            if (nb)
                HIPCHK(h, f64 ? launch_fixup<double>(c, A, B, h->lo.bead_off[b], nb, s_off)
                              : launch_fixup<float>(c, A, B, h->lo.bead_off[b], nb, s_off));
        }
    }
    return LB_OK;
}

// Batched coupled steps run as a pipeline with a step head when some large
// chain sits in a sparse box, no box is dense and the tiles are deferred.
bool headed_steps(const lb_handle* h)
{
    const Layout& lo = h->lo;
    return h->batched && h->overlap && lo.beads_big_sparse > 0 && lo.field_nodes == 0 && !h->ctx.keep_imp &&
           !h->ctx.tape;
}

// A run of n batched steps from buffer `from` (step offsets 0..n-1), on the
// two streams in turn.  Step k's plain collide runs on queue P[k & 1]; the
// other queue, right behind step k-1's collide, holds step k's chain work:
// the fix-up of the small chains' nodes of step k-1, the node-table kernel
// (which also re-collides step k-1's large-chain impulses outside its
// deferred tiles, and stamps step k's deferred tiles), then the chain kernel,
// the spread, the deferred tiles' list and collide, and the small chains'
// coupling.  Step k's collide waits for the node table only.  So the node
// table follows the previous collide on its own queue, and one short kernel
// separates two plain collides; the chain kernel, queued right behind the
// node table, starts before the collide it runs beside (it needs a whole CU,
// and its first reads are done before the collide loads the memory system).
// The run ends with the last step's leftovers and a join into the handle's
// stream.  Each node gets the same collide call with the same impulse as in
// enqueue_step, so the bits are the same.
lb_status enqueue_headed_run(lb_handle* h, int from, uint32_t n)
{
    const Layout& lo = h->lo;
    const bool f64 = h->prec == LB_FP64;
    LaunchCtx cq[2] = {h->ctx, h->ctx2};
    cq[0].defer_on = cq[1].defer_on = 1;
    hipStream_t P[2] = {h->stream, h->stream2};
    const int nc = (int)h->couple_host.size(), nbig = (int)lo.big_list.size();
    const bool small_fix = lo.beads_sparse > lo.beads_big_sparse;
    const uint32_t ts = (uint32_t)lo.tiles_sparse;
    const int one = nbig == 1 ? lo.big_list[0] : -1;
    HIPCHK(h, hipEventRecord(h->ev_fork, P[0]));
    HIPCHK(h, hipStreamWaitEvent(P[1], h->ev_fork, 0));
    for (uint32_t k = 0; k < n; ++k) {
        const int cqi = (int)(k & 1), wq = cqi ^ 1;   // collide queue, chain-work queue
        const LaunchCtx& cw = cq[wq];
        const int p = from ^ (int)(k & 1);
        const void* A = h->pop(p);
        void* B = h->pop(1 - p);
        // the previous step read pop(1 - p) and wrote pop(p)
        const void* prevA = h->pop(1 - p);
        void* prevB = h->pop(p);
        if (k > 0) {
            // step k-1's chain work (on this step's collide queue) is done
            HIPCHK(h, hipStreamWaitEvent(P[wq], h->ev_def, 0));
            if (small_fix)
                HIPCHK(h, f64 ? launch_fixup<double>(cw, prevA, prevB, 0, lo.total_beads, k - 1)
                              : launch_fixup<float>(cw, prevA, prevB, 0, lo.total_beads, k - 1));
        }
        const void* pend = k > 0 ? prevA : nullptr;
        HIPCHK(h, f64 ? launch_couple_big<double>(cw, A, h->big_list, nbig, lo.big_max_n, k, h->ev_head, pend, one)
                      : launch_couple_big<float>(cw, A, h->big_list, nbig, lo.big_max_n, k, h->ev_head, pend, one));
        if (nc)
            HIPCHK(h, f64 ? launch_couple<double>(cw, A, h->couple_list, nc, lo.couple_block, k)
                          : launch_couple<float>(cw, A, h->couple_list, nc, lo.couple_block, k));
        HIPCHK(h, f64 ? launch_collide_deferred<double>(cw, A, B, k) : launch_collide_deferred<float>(cw, A, B, k));
        HIPCHK(h, hipEventRecord(h->ev_def, P[wq]));
        HIPCHK(h, hipStreamWaitEvent(P[cqi], h->ev_head, 0));
        HIPCHK(h, f64 ? launch_collide<double>(cq[cqi], A, B, -1, 0, ts, k)
                      : launch_collide<float>(cq[cqi], A, B, -1, 0, ts, k));
    }
    // the last step's leftovers behind its collide, then everything joins
    // the handle's stream
    const int cl = (int)((n - 1) & 1);
    const int pl = from ^ (int)((n - 1) & 1);
    const void* lastA = h->pop(pl);
    void* lastB = h->pop(1 - pl);
    HIPCHK(h, hipStreamWaitEvent(P[cl], h->ev_def, 0));
    if (small_fix)
        HIPCHK(h, f64 ? launch_fixup<double>(cq[cl], lastA, lastB, 0, lo.total_beads, n - 1)
                      : launch_fixup<float>(cq[cl], lastA, lastB, 0, lo.total_beads, n - 1));
    HIPCHK(h, f64 ? launch_overflow<double>(cq[cl], lastA, lastB, n - 1)
                  : launch_overflow<float>(cq[cl], lastA, lastB, n - 1));
    if (cl == 1) {
        HIPCHK(h, hipEventRecord(h->ev_join, P[1]));
        HIPCHK(h, hipStreamWaitEvent(P[0], h->ev_join, 0));
    }
    return LB_OK;
}

// FP32 runs whose chains are all large (every box with beads holds a chain
// above BIG_CHAIN beads, none of them dense) take the collide that carries
// its own node tables from the second step on.  (In FP64 the node-table code
// would hold the collide to two waves per SIMD.)  Such runs rely on the two
// streams running on two hardware queues, so that the chain kernel of a step
// is resident before that step's collide: they are launched directly, never
// from a HIP graph, whose replay does not keep that order (the chain kernel's
// bounded wait then gives up).  A stream under capture takes the layout of
// enqueue_headed_run instead, and so does launch mode 3 (lb_set_launch), for
// tools that run one kernel at a time, such as hardware counter collection:
// there the waiting chain kernel can hold the GPU while the collide it waits
// for has not started.
// Batched coupled steps whose boxes hold chains of at most BIG_CHAIN beads
// and no dense box, with so few nodes that the collide (~30 us per million
// nodes in FP32) is shorter than the coupling kernel (a few us per MD
// substep): the chain's queue sets the step time.
constexpr uint64_t CHAIN_BOUND_NODES = 1ull << 20;
bool chain_bound_steps(const lb_handle* h)
{
    const Layout& lo = h->lo;
    return h->batched && h->overlap && !h->couple_host.empty() && lo.big_list.empty() && lo.field_nodes == 0 &&
           !h->ctx.keep_imp && !h->ctx.tape && lo.total_nodes <= CHAIN_BOUND_NODES;
}

// A run of n chain-bound steps from buffer `from` (step offsets 0..n-1),
// launched directly.  The second stream holds the chain work of one step
// after another: step k's coupling, then, once step k's collide is done, its
// fix-up.  The handle's stream holds the collides; step k's collide waits
// for step k-1's fix-up.  So the coupling kernels follow each other's
// fix-ups on one queue, and the collide beside each of them waits off that
// path (in the per-step form a coupling kernel waits for the previous
// fix-up on the other queue, and the fix-up for the coupling kernel).  A
// replayed graph maps its kernels onto queues of its own choosing, where
// the per-step form was measured faster, so a stream under capture takes
// that form.  Every node gets the same collide call with the same impulse
// as in enqueue_step, so the bits are the same.
lb_status enqueue_chain_run(lb_handle* h, int from, uint32_t n)
{
    const bool f64 = h->prec == LB_FP64;
    const LaunchCtx& c1 = h->ctx;
    const LaunchCtx& c2 = h->ctx2;
    const int nc = (int)h->couple_host.size();
    const uint32_t ts = (uint32_t)h->lo.tiles_sparse;
    HIPCHK(h, hipEventRecord(h->ev_fork, h->stream));
    HIPCHK(h, hipStreamWaitEvent(h->stream2, h->ev_fork, 0));
    for (uint32_t k = 0; k < n; ++k) {
        const int p = from ^ (int)(k & 1);
        const void* A = h->pop(p);
        void* B = h->pop(1 - p);
        // step k-1's fix-up wrote into A and read B
        if (k > 0) HIPCHK(h, hipStreamWaitEvent(h->stream, h->ev_join, 0));
        HIPCHK(h, f64 ? launch_collide<double>(c1, A, B, -1, 0, ts, k) : launch_collide<float>(c1, A, B, -1, 0, ts, k));
        HIPCHK(h, hipEventRecord(h->ev_coll, h->stream));
        HIPCHK(h, f64 ? launch_couple<double>(c2, A, h->couple_list, nc, h->lo.couple_block, k)
                      : launch_couple<float>(c2, A, h->couple_list, nc, h->lo.couple_block, k));
        HIPCHK(h, hipStreamWaitEvent(h->stream2, h->ev_coll, 0));
        if (h->lo.beads_sparse)
            HIPCHK(h, f64 ? launch_fixup<double>(c2, A, B, 0, h->lo.total_beads, k)
                          : launch_fixup<float>(c2, A, B, 0, h->lo.total_beads, k));
        HIPCHK(h, hipEventRecord(h->ev_join, h->stream2));
    }
    HIPCHK(h, hipStreamWaitEvent(h->stream, h->ev_join, 0));
    return LB_OK;
}

bool fused_steps(const lb_handle* h)
{
    // the collide's node-table workgroups wait for each other, so they must
    // fit on the GPU at once: at most one per CU
    return h->resident && headed_steps(h) && h->couple_host.empty() && h->prec == LB_FP32_DEV &&
           head_blocks((int)h->lo.big_list.size(), h->lo.big_max_n) <= (uint32_t)h->ctx.n_cu;
}

bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

// A run of n batched steps from buffer `from` in which every collide after
// the first carries the step's node tables.  The handle's stream holds the
// plain collides, the second stream the chain work, one step after another.
// Step 0 is laid out as in enqueue_step (node-table kernel, then the chain
// kernel and, once the table is there, the collide).  From step 1 on, step
// k's collide follows step k-1's collide and deferred tiles; its first
// workgroups fix up step k-1's impulses outside its deferred tiles and build
// step k's node tables.  Step k's chain kernel is queued behind step k-1's
// chain work, long before the previous collide ends: it gets a CU as that
// collide drains, before step k's collide starts, and waits there for the
// node-table workgroups.  Each chain kernel stamps the next step's deferred
// tiles from its end positions.  So a step is one collide and one kernel
// boundary.  Every node gets the same collide call with the same impulse as
// in enqueue_step, so the bits are the same.
lb_status enqueue_fused_run(lb_handle* h, int from, uint32_t n, uint32_t advance)
{
    const Layout& lo = h->lo;
    const bool f64 = h->prec == LB_FP64;
    LaunchCtx ca = h->ctx, cb = h->ctx2;
    ca.defer_on = cb.defer_on = 1;
    const int nbig = (int)lo.big_list.size();
    const uint32_t ts = (uint32_t)lo.tiles_sparse;
    const int one = nbig == 1 ? lo.big_list[0] : -1;
    const uint32_t n_head = head_blocks(nbig, lo.big_max_n);
    HIPCHK(h, hipEventRecord(h->ev_fork, h->stream));
    HIPCHK(h, hipStreamWaitEvent(h->stream2, h->ev_fork, 0));
    for (uint32_t k = 0; k < n; ++k) {
        const int p = from ^ (int)(k & 1);
        const void* A = h->pop(p);
        void* B = h->pop(1 - p);
        if (k == 0) {
            HIPCHK(h, f64 ? launch_couple_big<double>(cb, A, h->big_list, nbig, lo.big_max_n, 0, h->ev_head, nullptr,
                                                      one, 0, 1, 1)
                          : launch_couple_big<float>(cb, A, h->big_list, nbig, lo.big_max_n, 0, h->ev_head, nullptr,
                                                     one, 0, 1, 1));
            HIPCHK(h, hipStreamWaitEvent(h->stream, h->ev_head, 0));
            HIPCHK(h, f64 ? launch_collide<double>(ca, A, B, -1, 0, ts, 0) : launch_collide<float>(ca, A, B, -1, 0, ts, 0));
        } else {
            // step k-1 read pop(1 - p); its deferred tiles are collided
            HIPCHK(h, hipStreamWaitEvent(h->stream, h->ev_def, 0));
            const void* prevA = h->pop(1 - p);
            HIPCHK(h, f64 ? launch_collide_headed<double>(ca, A, B, ts, k, h->big_list, nbig, lo.big_max_n, prevA, one)
                          : launch_collide_headed<float>(ca, A, B, ts, k, h->big_list, nbig, lo.big_max_n, prevA, one));
            HIPCHK(h, f64 ? launch_couple_big<double>(cb, A, h->big_list, nbig, lo.big_max_n, k, nullptr, nullptr, one,
                                                      n_head, 0, 1)
                          : launch_couple_big<float>(cb, A, h->big_list, nbig, lo.big_max_n, k, nullptr, nullptr, one,
                                                     n_head, 0, 1));
        }
        HIPCHK(h, f64 ? launch_collide_deferred<double>(cb, A, B, k) : launch_collide_deferred<float>(cb, A, B, k));
        HIPCHK(h, hipEventRecord(h->ev_def, h->stream2));
    }
    // the last step's impulses outside its deferred tiles, then the counts
    // reset and the step counter advanced; the second stream has joined
    // through ev_def
    const int pl = from ^ (int)((n - 1) & 1);
    HIPCHK(h, hipStreamWaitEvent(h->stream, h->ev_def, 0));
    HIPCHK(h, f64 ? launch_overflow<double>(ca, h->pop(pl), h->pop(1 - pl), n - 1, advance)
                  : launch_overflow<float>(ca, h->pop(pl), h->pop(1 - pl), n - 1, advance));
    return LB_OK;
}

// n coupled steps from buffer `from`, step offsets 0..n-1, then the device
// step counter advanced by n
lb_status enqueue_steps(lb_handle* h, int from, uint32_t n)
{
    if (n == 0) return LB_OK;
    if (fused_steps(h) && !capturing(h->stream)) return enqueue_fused_run(h, from, n, n);
    if (headed_steps(h)) {
        const lb_status s = enqueue_headed_run(h, from, n);
        if (s != LB_OK) return s;
    } else if (chain_bound_steps(h) && !capturing(h->stream)) {
        const lb_status s = enqueue_chain_run(h, from, n);
        if (s != LB_OK) return s;
    } else {
        for (uint32_t k = 0; k < n; ++k) {
            const lb_status s = enqueue_step(h, from ^ (int)(k & 1), k, true);
            if (s != LB_OK) return s;
        }
    }
    HIPCHK(h, launch_advance(h->ctx, n));
    return LB_OK;
}

void drop_graphs(lb_handle* h)
{
    for (int p = 0; p < 2; ++p) {
        if (h->gexec[p]) (void)hipGraphExecDestroy(h->gexec[p]);
        if (h->graph[p]) (void)hipGraphDestroy(h->graph[p]);
        h->gexec[p] = nullptr;
        h->graph[p] = nullptr;
    }
}

lb_status build_graph(lb_handle* h, int parity)
{
    HIPCHK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    lb_status st = LB_OK;
    st = enqueue_steps(h, parity, (uint32_t)h->graph_steps);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->stream, &g);
    if (st != LB_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return fail(h, LB_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    h->graph[parity] = g;
    HIPCHK(h, hipGraphInstantiate(&h->gexec[parity], g, nullptr, nullptr, 0));
    return LB_OK;
}

// Record and instantiate the graphs of both buffer parities at once, so that
// no later lb_step captures or instantiates one (a caller timing lb_step
// then times replays only).  Synchronous.
lb_status prepare_graphs(lb_handle* h)
{
    drop_graphs(h);
    if (h->graph_steps <= 0 || fused_steps(h)) return LB_OK;
    for (int p = 0; p < 2; ++p) {
        lb_status s = build_graph(h, p);
        if (s != LB_OK) return s;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LB_OK;
}

}  // namespace

extern "C" {

lb_status lb_query_sizes(const lb_box_desc* boxes, int32_t n_boxes, int32_t precision, int32_t hist_steps,
                         size_t* state_bytes, size_t* scratch_bytes)
{
    std::string err;
    if (!validate(boxes, n_boxes, precision, hist_steps, err)) return fail(nullptr, LB_EINVAL, err);
    if (!state_bytes || !scratch_bytes) return fail(nullptr, LB_EINVAL, "null size pointer");
    Layout lo = make_layout(boxes, n_boxes, precision, hist_steps);
    *state_bytes = lo.state_bytes;
    *scratch_bytes = lo.scratch_bytes;
    return LB_OK;
}

lb_status lb_init(const lb_box_desc* boxes, int32_t n_boxes, int32_t precision, int32_t hist_steps,
                  const double* bead_x0, void* d_state, void* d_scratch, void* stream, lb_handle** out)
{
    std::string err;
    if (!out) return fail(nullptr, LB_EINVAL, "null handle pointer");
    *out = nullptr;
    if (!validate(boxes, n_boxes, precision, hist_steps, err)) return fail(nullptr, LB_EINVAL, err);
    if (!d_state || !d_scratch) return fail(nullptr, LB_EINVAL, "null device buffer");
    if (((uintptr_t)d_state & 255) || ((uintptr_t)d_scratch & 255))
        return fail(nullptr, LB_EINVAL, "device buffers must be 256-byte aligned");
    Layout lo = make_layout(boxes, n_boxes, precision, hist_steps);
    uint64_t nb = lo.total_beads;
    if (nb > 0 && !bead_x0) return fail(nullptr, LB_EINVAL, "bead_x0 is NULL but boxes have beads");
    // initial bonds (consecutive beads of one chain) must be shorter than R0
    for (int i = 0; i < n_boxes; ++i)
        for (int bd = 0; bd + 1 < boxes[i].n_beads; ++bd) {
            if (boxes[i].chain_len > 0 && (bd + 1) % boxes[i].chain_len == 0) continue;
            const double* p = bead_x0 + 3 * (lo.bead_off[i] + bd);
            double r2 = 0;
            for (int c = 0; c < 3; ++c) r2 += (p[3 + c] - p[c]) * (p[3 + c] - p[c]);
            if (!(r2 < boxes[i].r0_fene * boxes[i].r0_fene))
                return fail(nullptr, LB_EINVAL, "box " + std::to_string(i) + ": initial bond >= R0");
        }

    lb_handle* h = new lb_handle();
    h->n_boxes = n_boxes;
    h->prec = precision;
    h->hist = hist_steps;
    h->desc.assign(boxes, boxes + n_boxes);
    h->lo = lo;
    h->state = (char*)d_state;
    h->scratch = (char*)d_scratch;
    if (stream) {
        h->stream = (hipStream_t)stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) { delete h; return fail(nullptr, LB_EDEVICE, std::string("stream: ") + hipGetErrorString(e)); }
        h->own_stream = true;
    }
    auto sc = [&](size_t off) { return h->scratch + off; };
    auto stp = [&](size_t off) { return h->state + off; };

    std::vector<BoxDev> bd(n_boxes);
    for (int i = 0; i < n_boxes; ++i) {
        const lb_box_desc& d = boxes[i];
        BoxDev& b = bd[i];
        std::memset(&b, 0, sizeof b);
        b.L = d.L; b.N = d.n_beads; b.seed = d.seed; b.box_id = d.box_id;
        b.node_off = lo.node_off[i]; b.pop_off = lo.pop_off[i]; b.bead_off = lo.bead_off[i];
        b.tile_begin = lo.tile_begin[i]; b.n_tiles = lo.n_tiles[i];
        b.therm = d.thermalize; b.substeps = d.md_substeps;
        b.couple_T = lo.couple_T[i];
        b.chain_len = d.chain_len > 0 ? d.chain_len : std::max(d.n_beads, 1);
        b.dense = lo.dense[i];
        b.stat_off = lo.stat_off[i];
        b.field_off = lo.field_off[i];
        b.bin_off = lo.bin_off[i];
        b.item_off = lo.item_off[i];
        b.rho0 = d.rho0; b.gam_b = 1 - d.omega_bulk; b.gam_s = 1 - d.omega_shear; b.gam_g = 1 - d.omega_ghost;
        b.mu = 3.0 * d.kT * d.tau_lb * d.tau_lb;
        b.tau_lb = d.tau_lb; b.dt = d.md_dt; b.mass = d.bead_mass; b.zeta = d.zeta; b.k_fene = d.k_fene;
        b.r0sq = d.r0_fene * d.r0_fene; b.eps = d.eps_wca; b.sigsq = d.sigma_wca * d.sigma_wca;
        b.rc2 = std::pow(2.0, 1.0 / 3.0) * b.sigsq;
        b.bead_noise = std::sqrt(2.0 * d.kT * d.zeta / d.md_dt);
        b.inv_L = 1.0 / d.L;
        b.inv_r0sq = 1.0 / b.r0sq;
    }
    std::vector<uint32_t> tile_box(lo.total_tiles);
    for (int i = 0; i < n_boxes; ++i)
        for (uint32_t t = 0; t < lo.n_tiles[i]; ++t) tile_box[lo.tile_begin[i] + t] = (uint32_t)i;
    h->couple_host = lo.small_list;
    std::vector<int32_t> nlcnt(std::max<uint64_t>(nb, 1), -2);
    std::vector<int32_t> bead_box(std::max<uint64_t>(nb, 1), 0);
    for (int i = 0; i < n_boxes; ++i)
        for (int k = 0; k < boxes[i].n_beads; ++k) bead_box[lo.bead_off[i] + k] = i;

    auto up = [&](size_t off, const void* src, size_t bytes) {
        return bytes ? hipMemcpy(h->scratch + off, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    chk(hipMemsetAsync(h->scratch, 0, lo.scratch_bytes, h->stream));
    chk(hipMemsetAsync(h->state, 0, lo.state_bytes, h->stream));
    chk(hipStreamSynchronize(h->stream));
    chk(up(lo.sc_boxes, bd.data(), n_boxes * sizeof(BoxDev)));
    if (precision == LB_FP64) {
        std::vector<CollideConst<double>> cc(n_boxes);
        for (int i = 0; i < n_boxes; ++i) cc[i] = collide_const<double>(boxes[i]);
        chk(up(lo.sc_ccs, cc.data(), n_boxes * sizeof(cc[0])));
    } else {
        std::vector<CollideConst<float>> cc(n_boxes);
        for (int i = 0; i < n_boxes; ++i) cc[i] = collide_const<float>(boxes[i]);
        chk(up(lo.sc_ccs, cc.data(), n_boxes * sizeof(cc[0])));
    }
    chk(up(lo.sc_tilebox, tile_box.data(), tile_box.size() * sizeof(uint32_t)));
    chk(up(lo.sc_couple, h->couple_host.data(), h->couple_host.size() * sizeof(int32_t)));
    chk(up(lo.sc_beadbox, bead_box.data(), bead_box.size() * sizeof(int32_t)));
    chk(up(lo.sc_biglist, lo.big_list.data(), lo.big_list.size() * sizeof(int32_t)));
    chk(up(lo.sc_nlcnt, nlcnt.data(), nlcnt.size() * sizeof(int32_t)));
    if (nb) chk(hipMemcpy(stp(lo.st_x), bead_x0, nb * 3 * sizeof(double), hipMemcpyHostToDevice));
    if (e != hipSuccess) {
        std::string msg = std::string("init upload: ") + hipGetErrorString(e);
        lb_free(h);
        return fail(nullptr, LB_EDEVICE, msg);
    }

    LaunchCtx& c = h->ctx;
    c.stream = h->stream;
    {
        int dev = 0, ncu = 0;
        e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess || ncu <= 0) {
            std::string msg = std::string("device query: ") + hipGetErrorString(e);
            lb_free(h);
            return fail(nullptr, LB_EDEVICE, msg);
        }
        c.n_cu = ncu;
        c.collide_variant = DEFAULT_COLLIDE_VARIANT;
        h->dev = dev;
        h->static_scr = static_scratch(dev);   // once per device, this device current
    }
    c.boxes = (const BoxDev*)sc(lo.sc_boxes);
    h->boxes_host = bd;
    c.boxes_host = h->boxes_host.data();
    c.n_boxes = n_boxes;
    c.ccs = sc(lo.sc_ccs);
    c.tile_box = (const uint32_t*)sc(lo.sc_tilebox);
    c.ctrl = (Ctrl*)sc(lo.sc_ctrl);
    c.imp = (unsigned long long*)sc(lo.sc_imp);
    c.claim = (uint32_t*)sc(lo.sc_claim);
    c.touched = (uint32_t*)sc(lo.sc_touched);
    c.touched_cnt = (int32_t*)sc(lo.sc_tcnt);
    c.touch_cap = lo.touch_cap;
    c.nl_rebuilds = (uint32_t*)sc(lo.sc_nlreb);
    c.bead_box = (const int32_t*)sc(lo.sc_beadbox);
    c.x = (double*)stp(lo.st_x); c.v = (double*)stp(lo.st_v); c.f = (double*)stp(lo.st_f); c.fc = (double*)stp(lo.st_fc);
    c.nl_cnt = (int32_t*)sc(lo.sc_nlcnt); c.nl_idx = (uint16_t*)sc(lo.sc_nlidx); c.nl_x0 = (double*)sc(lo.sc_nlx0);
    c.nl_cap = NL_CAP;
    c.near_u = sc(lo.sc_nearu);
    c.near_c = (int4*)sc(lo.sc_nearc);
    c.field = sc(lo.sc_field);
    c.dense_max_tiles = lo.dense_max_tiles;
    c.big_sparse = 0;
    for (int i : lo.big_list) c.big_sparse += lo.dense[i] ? 0 : 1;
    c.bin_start = (uint32_t*)sc(lo.sc_binstart);
    c.runimp = (unsigned long long*)sc(lo.sc_items);
    c.slot_of = (uint32_t*)sc(lo.sc_slotof);
    c.sub_rec = (double*)sc(lo.sc_subrec);
    c.defer_on = 0;
    c.defer = (uint32_t*)sc(lo.sc_defer);
    c.dclaim = (uint32_t*)sc(lo.sc_dclaim);
    c.defer_list = (uint32_t*)sc(lo.sc_dlist);
    c.defer_cap = lo.defer_cap;
    c.ovf = (uint32_t*)sc(lo.sc_ovf);
    c.ovf_cap = lo.ovf_cap;
    c.ovm = (uint32_t*)sc(lo.sc_ovm);
    c.vhist = hist_steps > 0 ? (double*)sc(lo.sc_vhist) : nullptr;
    c.hist_len = hist_steps > 0 ? hist_steps : 1;
    c.total_beads = nb;
    h->couple_list = (int32_t*)sc(lo.sc_couple);
    h->big_list = (int32_t*)sc(lo.sc_biglist);
    e = hipStreamCreateWithFlags(&h->stream2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_table, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_head, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_def, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_coll, hipEventDisableTiming);
    if (e != hipSuccess) {
        std::string msg = std::string("second stream: ") + hipGetErrorString(e);
        lb_free(h);
        return fail(nullptr, LB_EDEVICE, msg);
    }
    h->ctx2 = c;
    h->ctx2.stream = h->stream2;

    {
        std::vector<int32_t> all;
        int mx = 0;
        for (int i = 0; i < n_boxes; ++i)
            if (boxes[i].n_beads > 0) { all.push_back(i); mx = std::max(mx, boxes[i].n_beads); }
        // every box with a chain
        int32_t* dl = (int32_t*)sc(lo.sc_alllist);
        e = all.empty() ? hipSuccess : hipMemcpy(dl, all.data(), all.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_init_forces(c, dl, (int)all.size(), std::max(64, (int)round_up((uint64_t)mx, 64)));
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        std::string msg = std::string("initial forces: ") + hipGetErrorString(e);
        lb_free(h);
        return fail(nullptr, LB_EDEVICE, msg);
    }
    *out = h;
    return LB_OK;
}

lb_status lb_couple(lb_handle* h)
{
    if (!h) return fail(nullptr, LB_EINVAL, "null handle");
    if (h->pending) return fail(h, LB_ESTATE, "lb_couple called twice without lb_step");
    {
        const void* A = h->pop(h->cur);
        const LaunchCtx& c = h->ctx;
        const int nc = (int)h->couple_host.size();
        const int nbig = (int)h->lo.big_list.size();
        if (nc) {
            if (h->prec == LB_FP64)
                HIPCHK(h, launch_couple<double>(c, A, h->couple_list, nc, h->lo.couple_block, 0));
            else
                HIPCHK(h, launch_couple<float>(c, A, h->couple_list, nc, h->lo.couple_block, 0));
        }
        if (nbig) {
            if (h->prec == LB_FP64)
                HIPCHK(h, launch_couple_big<double>(c, A, h->big_list, nbig, h->lo.big_max_n, 0, nullptr));
            else
                HIPCHK(h, launch_couple_big<float>(c, A, h->big_list, nbig, h->lo.big_max_n, 0, nullptr));
        }
    }
    h->pending = true;
    return LB_OK;
}

lb_status lb_step(lb_handle* h, int64_t n_steps)
{
    if (!h) return fail(nullptr, LB_EINVAL, "null handle");
    if (n_steps < 0) return fail(h, LB_EINVAL, "n_steps must be >= 0");
    int64_t left = n_steps;
    if (left > 0 && h->pending) {
        lb_status s = enqueue_step(h, h->cur, 0, false);
        if (s != LB_OK) return s;
        HIPCHK(h, launch_advance(h->ctx, 1));
        h->cur ^= 1;
        h->step += 1;
        h->pending = false;
        left -= 1;
    }
    if (h->graph_steps > 0 && !fused_steps(h)) {
        while (left >= h->graph_steps) {
            if (!h->gexec[h->cur]) {
                lb_status s = build_graph(h, h->cur);
                if (s != LB_OK) return s;
            }
            HIPCHK(h, hipGraphLaunch(h->gexec[h->cur], h->stream));
            left -= h->graph_steps;
            h->step += h->graph_steps;
        }
    }
    if (left > 0) {
        lb_status s = enqueue_steps(h, h->cur, (uint32_t)left);
        if (s != LB_OK) return s;
        if (left & 1) h->cur ^= 1;
        h->step += left;
    }
    return LB_OK;
}

}  // extern "C"

namespace {

// one box's lb_obs from its stats record s [NSTAT_REC] and chain record c
// [NCHAIN_REC]
void fill_obs(const lb_handle* h, int i, const double* s, const double* c, uint32_t rebuilds, const Ctrl& ctrl,
              lb_obs& o)
{
    const lb_box_desc& d = h->desc[i];
    std::memset(&o, 0, sizeof o);
    o.mass = (double)h->lo.V[i] * d.rho0 + s[0];
    for (int a = 0; a < 3; ++a) {
        o.j_lat[a] = s[1 + a];
        o.p_fluid[a] = s[1 + a] / d.tau_lb;
        o.p_beads[a] = c[3 + a];
        o.p_total[a] = o.p_fluid[a] + o.p_beads[a] + 0.5 * d.md_dt * c[6 + a];
        o.com[a] = d.n_beads > 0 ? c[a] / d.n_beads : 0.0;
    }
    // record: [9] sum over chains of R_e^2, [10] sum over beads of the
    // square distance to their chain's centre of mass
    const int chains = d.n_beads > 0 ? (d.chain_len > 0 ? d.n_beads / d.chain_len : 1) : 1;
    o.rg2 = d.n_beads > 0 ? c[10] / d.n_beads : 0.0;
    o.re2 = c[9] / chains;
    o.neg_count = s[4];
    for (int k = 0; k < 19; ++k) o.mode_sq[k] = s[5 + k];
    o.health = ctrl.health;
    o.nlist_builds = rebuilds;
    o.step = ctrl.step;
}

}  // namespace

extern "C" {

lb_status lb_observables(lb_handle* h, lb_obs* out)
{
    if (!h || !out) return fail(h, LB_EINVAL, "null argument");
    const Layout& lo = h->lo;
    double* part = (double*)(h->scratch + lo.sc_part);
    double* stat = (double*)(h->scratch + lo.sc_stat);
    double* chain = (double*)(h->scratch + lo.sc_chain);
    const void* A = h->pop(h->cur);
    double* mid = (double*)(h->scratch + lo.sc_mid);
    if (h->prec == LB_FP64)
        HIPCHK(h, launch_stats<double>(h->ctx, A, lo.stat_max_recs, part, mid, stat));
    else
        HIPCHK(h, launch_stats<float>(h->ctx, A, lo.stat_max_recs, part, mid, stat));
    HIPCHK(h, launch_chain_obs(h->ctx, chain));
    std::vector<double> st(h->n_boxes * NSTAT_REC), ch(h->n_boxes * NCHAIN_REC);
    std::vector<uint32_t> reb(h->n_boxes);
    Ctrl ctrl;
    HIPCHK(h, hipMemcpyAsync(reb.data(), h->scratch + lo.sc_nlreb, reb.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(st.data(), stat, st.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(ch.data(), chain, ch.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(&ctrl, h->scratch + lo.sc_ctrl, sizeof ctrl, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int i = 0; i < h->n_boxes; ++i)
        fill_obs(h, i, &st[i * NSTAT_REC], &ch[i * NCHAIN_REC], reb[i], ctrl, out[i]);
    if (ctrl.health) return fail(h, LB_ENUMERIC, "device health flags set: " + std::to_string(ctrl.health));
    return LB_OK;
}

lb_status lb_observables_static(lb_handle* h, lb_obs* out)
{
    if (!h || !out) return fail(h, LB_EINVAL, "null argument");
    if (!h->static_scr) return fail(h, LB_EDEVICE, "no device address for the static partial-sum array");
    const Layout& lo = h->lo;
    // partials in the static array: block records, chunk sums, box sums, chain records
    const size_t part_b = align256((size_t)lo.stat_recs * NSTAT_REC * sizeof(double));
    const size_t mid_b = align256((size_t)h->n_boxes * STAT_CHUNKS * NSTAT_REC * sizeof(double));
    const size_t stat_b = align256((size_t)h->n_boxes * NSTAT_REC * sizeof(double));
    const size_t chain_b = align256((size_t)h->n_boxes * NCHAIN_REC * sizeof(double));
    if (part_b + mid_b + stat_b + chain_b > STATIC_SCRATCH_BYTES)
        return fail(h, LB_ENOMEM, "boxes need " + std::to_string(part_b + mid_b + stat_b + chain_b) +
                                      " bytes of partial sums; the static array holds " +
                                      std::to_string(STATIC_SCRATCH_BYTES));
    char* base = (char*)h->static_scr;
    double* part = (double*)base;
    double* mid = (double*)(base + part_b);
    double* stat = (double*)(base + part_b + mid_b);
    double* chain = (double*)(base + part_b + mid_b + stat_b);
    const void* A = h->pop(h->cur);
    // every partial the kernels read is written earlier in the same call, so
    // no value carries over from a previous call
    if (h->prec == LB_FP64)
        HIPCHK(h, launch_stats<double>(h->ctx, A, lo.stat_max_recs, part, mid, stat));
    else
        HIPCHK(h, launch_stats<float>(h->ctx, A, lo.stat_max_recs, part, mid, stat));
    HIPCHK(h, launch_chain_obs(h->ctx, chain));
    Ctrl ctrl;
    HIPCHK(h, hipMemcpyAsync(&ctrl, h->scratch + lo.sc_ctrl, sizeof ctrl, hipMemcpyDeviceToHost, h->stream));
    // results to the host in chunks of boxes, through fixed buffers
    constexpr int CH = 32;
    double st[CH * NSTAT_REC], ch[CH * NCHAIN_REC];
    uint32_t reb[CH];
    for (int b0 = 0; b0 < h->n_boxes; b0 += CH) {
        const int nb = std::min(CH, h->n_boxes - b0);
        HIPCHK(h, hipMemcpyAsync(st, stat + (size_t)b0 * NSTAT_REC, (size_t)nb * NSTAT_REC * sizeof(double),
                                 hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipMemcpyAsync(ch, chain + (size_t)b0 * NCHAIN_REC, (size_t)nb * NCHAIN_REC * sizeof(double),
                                 hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipMemcpyAsync(reb, h->scratch + lo.sc_nlreb + (size_t)b0 * sizeof(uint32_t),
                                 (size_t)nb * sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        for (int i = 0; i < nb; ++i)
            fill_obs(h, b0 + i, &st[i * NSTAT_REC], &ch[i * NCHAIN_REC], reb[i], ctrl, out[b0 + i]);
    }
    if (ctrl.health) return fail(h, LB_ENUMERIC, "device health flags set: " + std::to_string(ctrl.health));
    return LB_OK;
}

size_t lb_state_host_bytes(const lb_handle* h)
{
    if (!h) return 0;
    size_t n = sizeof(uint64_t);
    for (int i = 0; i < h->n_boxes; ++i) n += (19 * h->lo.V[i] + 12 * (uint64_t)h->desc[i].n_beads) * sizeof(double);
    return n;
}

lb_status lb_export_state(lb_handle* h, void* host_buf, size_t bytes)
{
    if (!h || !host_buf) return fail(h, LB_EINVAL, "null argument");
    if (bytes < lb_state_host_bytes(h)) return fail(h, LB_ENOMEM, "host buffer too small");
    const Layout& lo = h->lo;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    Ctrl ctrl;
    HIPCHK(h, hipMemcpy(&ctrl, h->scratch + lo.sc_ctrl, sizeof ctrl, hipMemcpyDeviceToHost));
    char* o = (char*)host_buf;
    uint64_t stepv = ctrl.step;
    std::memcpy(o, &stepv, sizeof stepv);
    o += sizeof stepv;
    const char* P = (const char*)h->pop(h->cur);
    for (int i = 0; i < h->n_boxes; ++i) {
        const uint64_t V = lo.V[i];
        double* n = (double*)o;
        std::vector<char> raw(pop_elems_of(V) * lo.esz);
        const int L = h->desc[i].L;
        HIPCHK(h, hipMemcpy(raw.data(), P + lo.pop_off[i] * lo.esz, raw.size(), hipMemcpyDeviceToHost));
        for (int q = 0; q < 19; ++q) {
            const double base = wv(q) * h->desc[i].rho0;
            // stored p_q(s) is the population that arrives at s + c_q
            for (int z = 0; z < L; ++z)
                for (int y = 0; y < L; ++y)
                    for (int x = 0; x < L; ++x) {
                        const uint64_t s = x + (uint64_t)L * (y + (uint64_t)L * z);
                        const int xd = (x + cxv(q) + L) % L, yd = (y + cyv(q) + L) % L, zd = (z + czv(q) + L) % L;
                        const uint64_t dd = xd + (uint64_t)L * (yd + (uint64_t)L * zd);
                        const uint64_t a = pop_at(q, (uint32_t)s);
                        const double dv = lo.esz == 8 ? ((const double*)raw.data())[a] : (double)((const float*)raw.data())[a];
                        n[q * V + dd] = base + dv;
                    }
        }
        o += 19 * V * sizeof(double);
        const size_t nbb = (size_t)h->desc[i].n_beads * 3 * sizeof(double);
        const size_t goff = lo.bead_off[i] * 3 * sizeof(double);
        for (size_t arr : {lo.st_x, lo.st_v, lo.st_f, lo.st_fc}) {
            if (nbb) HIPCHK(h, hipMemcpy(o, h->state + arr + goff, nbb, hipMemcpyDeviceToHost));
            o += nbb;
        }
    }
    if (ctrl.health) return fail(h, LB_ENUMERIC, "device health flags set: " + std::to_string(ctrl.health));
    return LB_OK;
}

lb_status lb_import_state(lb_handle* h, const void* host_buf, size_t bytes)
{
    if (!h || !host_buf) return fail(h, LB_EINVAL, "null argument");
    if (bytes < lb_state_host_bytes(h)) return fail(h, LB_ENOMEM, "host buffer too small");
    if (h->pending) return fail(h, LB_ESTATE, "impulses pending from lb_couple");
    const Layout& lo = h->lo;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const char* o = (const char*)host_buf;
    uint64_t stepv;
    std::memcpy(&stepv, o, sizeof stepv);
    o += sizeof stepv;
    char* P = (char*)h->pop(h->cur);
    for (int i = 0; i < h->n_boxes; ++i) {
        const uint64_t V = lo.V[i];
        const double* n = (const double*)o;
        std::vector<char> raw(pop_elems_of(V) * lo.esz, 0);
        const int L = h->desc[i].L;
        for (int q = 0; q < 19; ++q) {
            const double base = wv(q) * h->desc[i].rho0;
            for (int z = 0; z < L; ++z)
                for (int y = 0; y < L; ++y)
                    for (int x = 0; x < L; ++x) {
                        const uint64_t s = x + (uint64_t)L * (y + (uint64_t)L * z);
                        const int xd = (x + cxv(q) + L) % L, yd = (y + cyv(q) + L) % L, zd = (z + czv(q) + L) % L;
                        const double dv = n[q * V + xd + (uint64_t)L * (yd + (uint64_t)L * zd)] - base;
                        const uint64_t a = pop_at(q, (uint32_t)s);
                        if (lo.esz == 8) ((double*)raw.data())[a] = dv;
                        else ((float*)raw.data())[a] = (float)dv;
                    }
        }
        HIPCHK(h, hipMemcpy(P + lo.pop_off[i] * lo.esz, raw.data(), raw.size(), hipMemcpyHostToDevice));
        o += 19 * V * sizeof(double);
        const size_t nbb = (size_t)h->desc[i].n_beads * 3 * sizeof(double);
        const size_t goff = lo.bead_off[i] * 3 * sizeof(double);
        for (size_t arr : {lo.st_x, lo.st_v, lo.st_f, lo.st_fc}) {
            if (nbb) HIPCHK(h, hipMemcpy(h->state + arr + goff, o, nbb, hipMemcpyHostToDevice));
            o += nbb;
        }
    }
    Ctrl ctrl;
    HIPCHK(h, hipMemcpy(&ctrl, h->scratch + lo.sc_ctrl, sizeof ctrl, hipMemcpyDeviceToHost));
    ctrl.step = (uint32_t)stepv;
    HIPCHK(h, hipMemcpy(h->scratch + lo.sc_ctrl, &ctrl, sizeof ctrl, hipMemcpyHostToDevice));
    std::vector<int32_t> nlcnt(std::max<uint64_t>(lo.total_beads, 1), -2);
    HIPCHK(h, hipMemcpy(h->scratch + lo.sc_nlcnt, nlcnt.data(), nlcnt.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    // fix-up claims and deferral stamps are step stamps: a restored step
    // count must not meet stale ones
    HIPCHK(h, clear_step_stamps(h));
    h->step = stepv;
    return LB_OK;
}

lb_status lb_pending_impulse(lb_handle* h, double* host_dense, size_t bytes)
{
    if (!h || !host_dense) return fail(h, LB_EINVAL, "null argument");
    const Layout& lo = h->lo;
    size_t need = 0;
    for (int i = 0; i < h->n_boxes; ++i) need += 3 * lo.V[i] * sizeof(double);
    if (bytes < need) return fail(h, LB_ENOMEM, "host buffer too small");
    std::memset(host_dense, 0, need);
    if (!lo.total_beads) return LB_OK;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    size_t base = 0;
    for (int i = 0; i < h->n_boxes; ++i) {
        const uint64_t V = lo.V[i];
        std::vector<unsigned long long> q(3 * V);
        HIPCHK(h, hipMemcpy(q.data(), h->scratch + lo.sc_imp + 3 * lo.node_off[i] * sizeof(unsigned long long),
                            q.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
        for (uint64_t r = 0; r < V; ++r)
            for (int c = 0; c < 3; ++c) host_dense[base + c * V + r] = (double)(long long)q[3 * r + c] * IMP_INV_SCALE;
        base += 3 * V;
    }
    return LB_OK;
}

lb_status lb_velocity_history(lb_handle* h, int64_t step, double* host_out, size_t bytes)
{
    if (!h || !host_out) return fail(h, LB_EINVAL, "null argument");
    if (h->hist <= 0) return fail(h, LB_ESTATE, "no velocity history was requested at init");
    const uint64_t nb = h->lo.total_beads;
    if (bytes < nb * 3 * sizeof(double)) return fail(h, LB_ENOMEM, "host buffer too small");
    const int64_t now = (int64_t)h->step;
    if (step < 0 || step >= now || step < now - h->hist) return fail(h, LB_EINVAL, "step not in the history ring");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    const size_t off = h->lo.sc_vhist + (size_t)(step % h->hist) * nb * 3 * sizeof(double);
    HIPCHK(h, hipMemcpy(host_out, h->scratch + off, nb * 3 * sizeof(double), hipMemcpyDeviceToHost));
    return LB_OK;
}

lb_status lb_bead_positions(lb_handle* h, double* host_out, size_t bytes)
{
    if (!h || !host_out) return fail(h, LB_EINVAL, "null argument");
    const uint64_t nb = h->lo.total_beads;
    if (bytes < nb * 3 * sizeof(double)) return fail(h, LB_ENOMEM, "host buffer too small");
    if (h->pending) return fail(h, LB_ESTATE, "impulses pending from lb_couple");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (nb) HIPCHK(h, hipMemcpy(host_out, h->state + h->lo.st_x, nb * 3 * sizeof(double), hipMemcpyDeviceToHost));
    return LB_OK;
}

lb_status lb_set_launch(lb_handle* h, int32_t batched, int32_t graph_steps)
{
    if (!h) return fail(nullptr, LB_EINVAL, "null handle");
    if (graph_steps < 0) return fail(h, LB_EINVAL, "graph_steps must be >= 0");
    if (batched < 0 || batched > 3) return fail(h, LB_EINVAL, "batched must be 0, 1, 2 or 3");
    if (h->pending) return fail(h, LB_ESTATE, "impulses pending from lb_couple");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    drop_graphs(h);
    h->batched = batched ? 1 : 0;
    h->overlap = batched == 2 ? 0 : 1;
    h->resident = batched == 3 ? 0 : 1;
    h->graph_steps = graph_steps + (graph_steps & 1);
    return prepare_graphs(h);
}


}  // extern "C"

// ------------------------------------------------------------ adjoint window
namespace {

// Two tape sets (populations, impulses, substep records, starting beads of
// each step of a segment): the backward replays one segment into one set
// while it reverses the previously replayed segment from the other.
struct WinLayout {
    size_t ck_pop, ck_beads, tape_pop[2], tape_imp[2], tape_sub[2], tape_beads[2], vh, dj, lam_a, lam_b, lam_dp,
        lbeads, gpart, gz, bytes;
    size_t bspan;   // bytes of the state's x, v, f arrays, gaps included
    int nc;
};

WinLayout win_layout(const lb_handle* h, int T, int k)
{
    const Layout& lo = h->lo;
    WinLayout w{};
    const uint64_t nb = std::max<uint64_t>(lo.total_beads, 1), nodes = lo.total_nodes;
    const size_t popb = lo.pop_elems * lo.esz;
    int smax = 1;
    for (const auto& d : h->desc) smax = std::max(smax, d.md_substeps);
    w.nc = (T + k - 1) / k;
    size_t o = 0;
    w.ck_pop = o; o = align256(o + (size_t)(w.nc + 1) * popb);
    w.ck_beads = o; o = align256(o + (size_t)(w.nc + 1) * 12 * nb * sizeof(double));
    w.bspan = lo.st_fc - lo.st_x;   // x, v, f of the state, with their alignment gaps
    for (int b = 0; b < 2; ++b) {
        w.tape_pop[b] = o; o = align256(o + (size_t)(k + 1) * popb);
        w.tape_imp[b] = o; o = align256(o + (size_t)k * 3 * nodes * sizeof(unsigned long long));
        w.tape_sub[b] = o; o = align256(o + (size_t)k * smax * nb * TAPE_REC * sizeof(double));
        w.tape_beads[b] = o; o = align256(o + (size_t)k * w.bspan);
    }
    w.vh = o; o = align256(o + (size_t)T * 3 * nb * sizeof(double));
    w.dj = o; o = align256(o + (size_t)T * 3 * nb * sizeof(double));
    w.lam_a = o; o = align256(o + 19 * nodes * sizeof(double));
    w.lam_b = o; o = align256(o + 19 * nodes * sizeof(double));
    w.lam_dp = o; o = align256(o + 3 * nodes * sizeof(double));
    w.lbeads = o; o = align256(o + 9 * nb * sizeof(double));
    w.gpart = o; o = align256(o + 2 * lo.total_tiles * sizeof(double));
    w.gz = o; o = align256(o + h->n_boxes * sizeof(double));
    w.bytes = o;
    return w;
}

// copy the current state (pops of the current buffer, beads) into / out of slot j
lb_status ck_save(lb_handle* h, char* ws, const WinLayout& w, int j)
{
    const Layout& lo = h->lo;
    const size_t popb = lo.pop_elems * lo.esz, bb = 3 * std::max<uint64_t>(lo.total_beads, 1) * sizeof(double);
    HIPCHK(h, hipMemcpyAsync(ws + w.ck_pop + j * popb, h->pop(h->cur), popb, hipMemcpyDeviceToDevice, h->stream));
    char* dst = ws + w.ck_beads + (size_t)j * 4 * bb;
    const size_t arrs[4] = {lo.st_x, lo.st_v, lo.st_f, lo.st_fc};
    for (int a = 0; a < 4; ++a)
        HIPCHK(h, hipMemcpyAsync(dst + a * bb, h->state + arrs[a], bb, hipMemcpyDeviceToDevice, h->stream));
    return LB_OK;
}

// enqueue on the main stream the copy of slot j's beads into the state
lb_status ck_restore_beads(lb_handle* h, char* ws, const WinLayout& w, int j)
{
    const Layout& lo = h->lo;
    const size_t bb = 3 * std::max<uint64_t>(lo.total_beads, 1) * sizeof(double);
    const char* src = ws + w.ck_beads + (size_t)j * 4 * bb;
    const size_t arrs[4] = {lo.st_x, lo.st_v, lo.st_f, lo.st_fc};
    for (int a = 0; a < 4; ++a)
        HIPCHK(h, hipMemcpyAsync(h->state + arrs[a], src + a * bb, bb, hipMemcpyDeviceToDevice, h->stream));
    return LB_OK;
}

// set the device step counter (the main stream is drained first)
lb_status set_device_step(lb_handle* h, uint64_t step)
{
    const Layout& lo = h->lo;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    Ctrl ctrl;
    HIPCHK(h, hipMemcpy(&ctrl, h->scratch + lo.sc_ctrl, sizeof ctrl, hipMemcpyDeviceToHost));
    ctrl.step = (uint32_t)step;
    HIPCHK(h, hipMemcpy(h->scratch + lo.sc_ctrl, &ctrl, sizeof ctrl, hipMemcpyHostToDevice));
    return LB_OK;
}

lb_status ck_restore(lb_handle* h, char* ws, const WinLayout& w, int j, uint64_t step)
{
    const Layout& lo = h->lo;
    const size_t popb = lo.pop_elems * lo.esz;
    h->cur = 0;
    HIPCHK(h, hipMemcpyAsync(h->pop(0), ws + w.ck_pop + j * popb, popb, hipMemcpyDeviceToDevice, h->stream));
    lb_status s = ck_restore_beads(h, ws, w, j);
    if (s == LB_OK) s = set_device_step(h, step);
    if (s != LB_OK) return s;
    HIPCHK(h, clear_step_stamps(h));
    h->step = step;
    return LB_OK;
}

// One LB step of a window from populations A into B, its launches serialised
// on the main stream: step number = device step counter + s_off (the caller
// advances the counter once after a run of steps).  imp: where the node
// impulses go (null: the library's field, consumed by the fix-up; else a
// zeroed tape slot that keeps them); tape: substep tape (null: none), with
// tape_beads the step's starting x, v, f in the state's layout; vh, hist_len:
// ring of bead velocities after each step (null: the handle's own).
lb_status window_step(lb_handle* h, const void* A, void* B, unsigned long long* imp, double* tape,
                      double* tape_beads, double* vh, int hist_len, uint32_t s_off)
{
    const bool f64 = h->prec == LB_FP64;
    LaunchCtx c = h->ctx;
    c.tape = tape;
    c.tape_x0 = tape ? tape_beads : nullptr;
    c.tape_vo = (h->lo.st_v - h->lo.st_x) / sizeof(double);
    c.tape_fo = (h->lo.st_f - h->lo.st_x) / sizeof(double);
    if (imp) { c.imp = imp; c.keep_imp = 1; }
    if (vh) { c.vhist = vh; c.hist_len = hist_len; }
    const int nc = (int)h->couple_host.size();
    if (nc)
        HIPCHK(h, f64 ? launch_couple<double>(c, A, h->couple_list, nc, h->lo.couple_block, s_off)
                      : launch_couple<float>(c, A, h->couple_list, nc, h->lo.couple_block, s_off));
    HIPCHK(h, f64 ? launch_collide<double>(c, A, B, -1, 0, (uint32_t)h->lo.total_tiles, s_off)
                  : launch_collide<float>(c, A, B, -1, 0, (uint32_t)h->lo.total_tiles, s_off));
    if (h->lo.total_beads)
        HIPCHK(h, f64 ? launch_fixup<double>(c, A, B, 0, h->lo.total_beads, s_off)
                      : launch_fixup<float>(c, A, B, 0, h->lo.total_beads, s_off));
    h->step += 1;
    return LB_OK;
}

}  // namespace

extern "C" {

size_t lb_window_bytes(const lb_handle* h, int32_t T, int32_t k)
{
    if (!h || T <= 0 || k <= 0) return 0;
    return win_layout(h, T, std::min(k, T)).bytes;
}

lb_status lb_set_rates(lb_handle* h, int32_t box, double omega_shear, double omega_bulk, double zeta)
{
    if (!h) return fail(nullptr, LB_EINVAL, "null handle");
    if (box < 0 || box >= h->n_boxes) return fail(h, LB_EINVAL, "box index out of range");
    if (!(omega_shear > 0 && omega_shear < 2) || !(omega_bulk > 0 && omega_bulk < 2) || !(zeta >= 0))
        return fail(h, LB_EINVAL, "rates out of range");
    if (h->pending) return fail(h, LB_ESTATE, "impulses pending from lb_couple");
    lb_box_desc& d = h->desc[box];
    d.omega_shear = omega_shear;
    d.omega_bulk = omega_bulk;
    d.zeta = zeta;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    BoxDev b;
    HIPCHK(h, hipMemcpy(&b, h->scratch + h->lo.sc_boxes + box * sizeof(BoxDev), sizeof b, hipMemcpyDeviceToHost));
    b.gam_b = 1 - omega_bulk;
    b.gam_s = 1 - omega_shear;
    b.zeta = zeta;
    b.bead_noise = std::sqrt(2.0 * d.kT * zeta / d.md_dt);
    HIPCHK(h, hipMemcpy(h->scratch + h->lo.sc_boxes + box * sizeof(BoxDev), &b, sizeof b, hipMemcpyHostToDevice));
    h->boxes_host[box] = b;   // launches that pass a descriptor by value are recorded again below
    if (h->prec == LB_FP64) {
        CollideConst<double> cc = collide_const<double>(d);
        HIPCHK(h, hipMemcpy(h->scratch + h->lo.sc_ccs + box * sizeof(cc), &cc, sizeof cc, hipMemcpyHostToDevice));
    } else {
        CollideConst<float> cc = collide_const<float>(d);
        HIPCHK(h, hipMemcpy(h->scratch + h->lo.sc_ccs + box * sizeof(cc), &cc, sizeof cc, hipMemcpyHostToDevice));
    }
    return prepare_graphs(h);
}

lb_status lb_window_forward(lb_handle* h, void* d_ws, size_t bytes, int32_t T, int32_t k, double* vhist_host)
{
    if (!h || !d_ws) return fail(h, LB_EINVAL, "null argument");
    if (T <= 0 || k <= 0) return fail(h, LB_EINVAL, "T and k must be positive");
    if (h->pending) return fail(h, LB_ESTATE, "impulses pending from lb_couple");
    if (!h->lo.big_list.empty()) return fail(h, LB_EINVAL, "the adjoint window supports chains of at most 256 beads");
    k = std::min(k, T);
    const WinLayout w = win_layout(h, T, k);
    if (bytes < w.bytes) return fail(h, LB_ENOMEM, "window workspace too small");
    char* ws = (char*)d_ws;
    const uint64_t nb3 = 3 * std::max<uint64_t>(h->lo.total_beads, 1);
    h->win_T = T;
    h->win_k = k;
    h->win_step0 = h->step;
    // the coupling kernel writes the bead velocities after step s into slot
    // s mod T of the window's ring: slot (step0 + t) mod T holds step t
    int t_adv = 0;   // steps the device counter has been advanced by
    for (int t = 0; t < T; ++t) {
        if (t % k == 0) {
            lb_status s = ck_save(h, ws, w, t / k);
            if (s != LB_OK) return s;
        }
        lb_status s = window_step(h, h->pop(h->cur), h->pop(1 - h->cur), nullptr, nullptr, nullptr,
                                  (double*)(ws + w.vh), T, (uint32_t)(t - t_adv));
        if (s != LB_OK) return s;
        h->cur ^= 1;
        if ((t + 1) % k == 0 || t + 1 == T) {   // the device counter catches up before a checkpoint
            HIPCHK(h, launch_advance(h->ctx, (uint32_t)(t + 1 - t_adv)));
            t_adv = t + 1;
        }
    }
    if (vhist_host) {
        std::vector<double> ring((size_t)T * nb3);
        HIPCHK(h, hipMemcpyAsync(ring.data(), ws + w.vh, ring.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
        const uint64_t r0 = h->win_step0 % (uint64_t)T;
        for (int t = 0; t < T; ++t)
            std::memcpy(vhist_host + (size_t)t * nb3, ring.data() + ((r0 + t) % T) * nb3, nb3 * sizeof(double));
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->win_ready = true;
    return LB_OK;
}

lb_status lb_window_rewind(lb_handle* h, void* d_ws, size_t bytes)
{
    if (!h || !d_ws) return fail(h, LB_EINVAL, "null argument");
    if (!h->win_ready) return fail(h, LB_ESTATE, "no forward window recorded");
    const WinLayout w = win_layout(h, h->win_T, h->win_k);
    if (bytes < w.bytes) return fail(h, LB_ENOMEM, "window workspace too small");
    return ck_restore(h, (char*)d_ws, w, 0, h->win_step0);
}

lb_status lb_window_backward(lb_handle* h, void* d_ws, size_t bytes, const double* dj_host, double* grad_host)
{
    if (!h || !d_ws || !dj_host || !grad_host) return fail(h, LB_EINVAL, "null argument");
    if (!h->win_ready) return fail(h, LB_ESTATE, "no forward window recorded");
    const int T = h->win_T, k = h->win_k;
    const WinLayout w = win_layout(h, T, k);
    if (bytes < w.bytes) return fail(h, LB_ENOMEM, "window workspace too small");
    char* ws = (char*)d_ws;
    const Layout& lo = h->lo;
    const uint64_t nbx = std::max<uint64_t>(lo.total_beads, 1), nb3 = 3 * nbx, nodes = lo.total_nodes;
    const size_t popb = lo.pop_elems * lo.esz;
    int smax = 1;
    for (const auto& d : h->desc) smax = std::max(smax, d.md_substeps);
    const bool f64 = h->prec == LB_FP64;
    // the reverse sweep works in FP64 whatever the storage precision
    if (!h->ccd) HIPCHK(h, hipMalloc(&h->ccd, h->n_boxes * sizeof(CollideConst<double>)));
    {
        std::vector<CollideConst<double>> cc(h->n_boxes);
        for (int i = 0; i < h->n_boxes; ++i) cc[i] = collide_const<double>(h->desc[i]);
        HIPCHK(h, hipMemcpy(h->ccd, cc.data(), cc.size() * sizeof(cc[0]), hipMemcpyHostToDevice));
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream2));
    // keep the end-of-window state, restored at the end
    lb_status st = ck_save(h, ws, w, w.nc);
    if (st != LB_OK) return st;
    const uint64_t step_end = h->step;
    const int cur_end = h->cur;
    // The segments are replayed on the main stream and reversed on the second
    // one: the replay of segment s - 1 (into one tape set) runs while segment
    // s is reversed (from the other).  The reverse kernels read only the tape,
    // the adjoint fields and the box tables, never the live state the replay
    // advances.
    hipStream_t rs = h->stream2;
    LaunchCtx rc = h->ctx2;
    struct Events {
        hipEvent_t e[4] = {};
        ~Events() { for (hipEvent_t x : e) if (x) (void)hipEventDestroy(x); }
    } ev;
    for (hipEvent_t& x : ev.e) HIPCHK(h, hipEventCreateWithFlags(&x, hipEventDisableTiming));
    hipEvent_t* replayed = ev.e;      // per tape set: its segment is recorded
    hipEvent_t* reversed = ev.e + 2;  // per tape set: its segment is reversed, the set is free
    bool in_use[2] = {false, false};
    HIPCHK(h, hipMemcpyAsync(ws + w.dj, dj_host, (size_t)T * nb3 * sizeof(double), hipMemcpyHostToDevice, rs));
    HIPCHK(h, hipMemsetAsync(ws + w.lam_a, 0, 19 * nodes * sizeof(double), rs));
    HIPCHK(h, hipMemsetAsync(ws + w.lam_b, 0, 19 * nodes * sizeof(double), rs));
    HIPCHK(h, hipMemsetAsync(ws + w.lbeads, 0, 9 * nbx * sizeof(double), rs));
    HIPCHK(h, hipMemsetAsync(ws + w.gpart, 0, 2 * lo.total_tiles * sizeof(double), rs));
    HIPCHK(h, hipMemsetAsync(ws + w.gz, 0, h->n_boxes * sizeof(double), rs));
    double* lam_next = (double*)(ws + w.lam_a);
    double* lam_cur = (double*)(ws + w.lam_b);
    double* lb = (double*)(ws + w.lbeads);
    // the device step counter stays at the window's first step; each replayed
    // step passes its offset in the window
    st = set_device_step(h, h->win_step0);
    if (st != LB_OK) return st;
    for (int seg = w.nc - 1; seg >= 0; --seg) {
        const int t0 = seg * k, t1 = std::min(T, t0 + k), tb = seg & 1;
        char* tpop = ws + w.tape_pop[tb];
        char* timp = ws + w.tape_imp[tb];
        char* tsub = ws + w.tape_sub[tb];
        char* tbeads = ws + w.tape_beads[tb];
        st = ck_restore_beads(h, ws, w, seg);
        if (st != LB_OK) return st;
        HIPCHK(h, clear_step_stamps(h, false));
        // the set was last read by the reverse of segment seg + 2
        if (in_use[tb]) HIPCHK(h, hipStreamWaitEvent(h->stream, reversed[tb], 0));
        // replay the segment, recording what the reverse sweep needs: step j
        // reads tape slot j and writes slot j + 1, and adds its impulses into
        // its own zeroed impulse slot
        HIPCHK(h, hipMemcpyAsync(tpop, ws + w.ck_pop + seg * popb, popb, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(h, hipMemsetAsync(timp, 0, (size_t)(t1 - t0) * 3 * nodes * 8, h->stream));
        for (int t = t0; t < t1; ++t) {
            const int j = t - t0;
            // the coupling kernel records the step's starting beads in slot j
            st = window_step(h, tpop + j * popb, tpop + (j + 1) * popb,
                             (unsigned long long*)(timp + (size_t)j * 3 * nodes * 8),
                             (double*)(tsub + (size_t)j * smax * nbx * TAPE_REC * sizeof(double)),
                             (double*)(tbeads + (size_t)j * w.bspan), nullptr, 0, (uint32_t)t);
            if (st != LB_OK) return st;
        }
        HIPCHK(h, hipEventRecord(replayed[tb], h->stream));
        HIPCHK(h, hipStreamWaitEvent(rs, replayed[tb], 0));
        // reverse the segment's steps
        for (int t = t1 - 1; t >= t0; --t) {
            const int j = t - t0;
            const uint32_t stepv = (uint32_t)(h->win_step0 + t);
            const char* P = tpop + j * popb;
            const unsigned long long* imp = (const unsigned long long*)(timp + (size_t)j * 3 * nodes * 8);
            HIPCHK(h, f64 ? launch_adj_collide<double>(rc, h->ccd, P, imp, lam_next, lam_cur,
                                                       (double*)(ws + w.lam_dp), (double*)(ws + w.gpart), nodes,
                                                       (uint32_t)lo.total_tiles, stepv)
                          : launch_adj_collide<float>(rc, h->ccd, P, imp, lam_next, lam_cur,
                                                      (double*)(ws + w.lam_dp), (double*)(ws + w.gpart), nodes,
                                                      (uint32_t)lo.total_tiles, stepv));
            AdjArgsHost a;
            const char* bj = tbeads + (size_t)j * w.bspan;   // x, v, f as laid out in the state
            a.x0 = (const double*)bj;
            a.v0 = (const double*)(bj + (lo.st_v - lo.st_x));
            a.f0 = (const double*)(bj + (lo.st_f - lo.st_x));
            a.tape = (const double*)(tsub + (size_t)j * smax * nbx * TAPE_REC * sizeof(double));
            a.dj = (const double*)(ws + w.dj) + (size_t)t * nb3;
            a.lx = lb; a.lv = lb + nb3; a.lf = lb + 2 * nb3;
            a.lam_n = lam_cur;
            a.lam_dp = (const double*)(ws + w.lam_dp);
            a.gz = (double*)(ws + w.gz);
            a.nodes = nodes;
            const int nc = (int)h->couple_host.size();
            HIPCHK(h, f64 ? launch_adj_couple<double>(rc, h->couple_list, nc, lo.couple_block, P, a, stepv)
                          : launch_adj_couple<float>(rc, h->couple_list, nc, lo.couple_block, P, a, stepv));
            std::swap(lam_next, lam_cur);
        }
        HIPCHK(h, hipEventRecord(reversed[tb], rs));
        in_use[tb] = true;
    }
    std::vector<double> gpart(2 * lo.total_tiles), gz(h->n_boxes);
    HIPCHK(h, hipMemcpyAsync(gpart.data(), ws + w.gpart, gpart.size() * sizeof(double), hipMemcpyDeviceToHost, rs));
    HIPCHK(h, hipMemcpyAsync(gz.data(), ws + w.gz, gz.size() * sizeof(double), hipMemcpyDeviceToHost, rs));
    HIPCHK(h, hipStreamSynchronize(rs));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int i = 0; i < h->n_boxes; ++i) {
        double gs = 0.0, gb = 0.0;
        for (uint32_t t = 0; t < lo.n_tiles[i]; ++t) {
            gs += gpart[2 * (lo.tile_begin[i] + t)];
            gb += gpart[2 * (lo.tile_begin[i] + t) + 1];
        }
        grad_host[3 * i] = gs;
        grad_host[3 * i + 1] = gb;
        grad_host[3 * i + 2] = gz[i];
    }
    // back to the end of the window
    st = ck_restore(h, ws, w, w.nc, step_end);
    if (st != LB_OK) return st;
    if (cur_end != 0) {   // the restored state sits in buffer 0; keep the handle's parity convention
        HIPCHK(h, hipMemcpyAsync(h->pop(1), h->pop(0), popb, hipMemcpyDeviceToDevice, h->stream));
        h->cur = 1;
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LB_OK;
}

}  // extern "C"

extern "C" {
lb_status lb_collide_only(lb_handle* h, int32_t n)
{
    if (!h) return fail(nullptr, LB_EINVAL, "null handle");
    if (n < 0) return fail(h, LB_EINVAL, "n must be >= 0");
    const void* A = h->pop(h->cur);
    void* B = h->pop(1 - h->cur);
    for (int32_t k = 0; k < n; ++k) {
        if (h->prec == LB_FP64)
            HIPCHK(h, launch_collide<double>(h->ctx, A, B, -1, 0, (uint32_t)h->lo.total_tiles, 0));
        else
            HIPCHK(h, launch_collide<float>(h->ctx, A, B, -1, 0, (uint32_t)h->lo.total_tiles, 0));
    }
    return LB_OK;
}

static_assert(LB_N_COLLIDE_VARIANTS == N_COLLIDE_VARIANTS, "variant count");

lb_status lb_set_collide_variant(lb_handle* h, int32_t variant)
{
    if (!h) return fail(nullptr, LB_EINVAL, "null handle");
    if (variant < 0 || variant >= N_COLLIDE_VARIANTS) return fail(h, LB_EINVAL, "variant out of range");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    h->ctx.collide_variant = h->ctx2.collide_variant = variant;
    return prepare_graphs(h);
}

lb_status lb_autotune(lb_handle* h, int32_t reps, float* times_us, int32_t* chosen)
{
    if (!h) return fail(nullptr, LB_EINVAL, "null handle");
    if (reps <= 0) return fail(h, LB_EINVAL, "reps must be > 0");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    drop_graphs(h);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(h, hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    bool launch_failed = false;    // lb_collide_only already set the message
    float best = 0.f;
    int best_v = h->ctx.collide_variant;
    const int keep = h->ctx.collide_variant;
    // two sweeps over the variants, each keeping its faster one: the first
    // launches after a pause run at lower clocks, which would otherwise
    // penalise whichever variant is timed first
    float tmin[N_COLLIDE_VARIANTS];
    for (int pass = 0; pass < 2 && e == hipSuccess && !launch_failed; ++pass) {
        for (int v = 0; v < N_COLLIDE_VARIANTS; ++v) {
            h->ctx.collide_variant = v;
            if (lb_collide_only(h, 2) != LB_OK) { launch_failed = true; break; }
            e = hipEventRecord(e0, h->stream);
            if (e != hipSuccess) break;
            if (lb_collide_only(h, reps) != LB_OK) { launch_failed = true; break; }
            e = hipEventRecord(e1, h->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) break;
            const float us = 1e3f * ms / reps;
            tmin[v] = pass == 0 ? us : std::min(tmin[v], us);
        }
    }
    if (e == hipSuccess && !launch_failed) {
        for (int v = 0; v < N_COLLIDE_VARIANTS; ++v) {
            if (times_us) times_us[v] = tmin[v];
            if (v == 0 || tmin[v] < best) { best = tmin[v]; best_v = v; }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (launch_failed || e != hipSuccess) {
        h->ctx.collide_variant = keep;
        if (!launch_failed) h->err = std::string("autotune: ") + hipGetErrorString(e);
        return LB_EDEVICE;
    }
    h->ctx.collide_variant = h->ctx2.collide_variant = best_v;
    if (chosen) *chosen = best_v;
    return prepare_graphs(h);
}

void* lb_stream(const lb_handle* h) { return h ? (void*)h->stream : nullptr; }

void lb_free(lb_handle* h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->stream2) (void)hipStreamSynchronize(h->stream2);
    drop_graphs(h);
    if (h->ccd) (void)hipFree(h->ccd);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    if (h->ev_table) (void)hipEventDestroy(h->ev_table);
    if (h->ev_head) (void)hipEventDestroy(h->ev_head);
    if (h->ev_def) (void)hipEventDestroy(h->ev_def);
    if (h->ev_coll) (void)hipEventDestroy(h->ev_coll);
    if (h->stream2) (void)hipStreamDestroy(h->stream2);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

const char* lb_last_error(const lb_handle* h) { return h ? h->err.c_str() : g_err.c_str(); }

}  // extern "C"
