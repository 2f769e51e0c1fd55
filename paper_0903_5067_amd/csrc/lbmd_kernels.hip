// HIP kernels of the fluctuating D3Q19 LB step with a dissipatively coupled
// bead-spring chain, for gfx950 (MI355X).
//
//   k_couple      chains of up to 256 beads, one workgroup per chain (T lanes
//                 per bead, T a function of N only): velocity-Verlet
//                 substeps in the fluid velocity field frozen at the
//                 pre-collision state, trilinear interpolation, friction +
//                 Langevin force, and the impulse handed back to the stencil
//                 nodes (Sec. II.B, coupling paragraph; potentials of
//                 Sec. II.A).  Impulses go into a dense fixed-point field by
//                 atomic adds that nothing waits on (order-independent, hence
//                 bitwise reproducible); each bead lists the nodes it touched.
//   k_collide     fused stream + collide of every node, no impulse
//                 (Sec. II.B, LB equation), thread per node; populations in
//                 1024-node tiles of 19 planes each (pop_at).
//                 Pull form: a buffer holds post-collision populations p,
//                 the pre-collision population of node r is n_i(r) =
//                 p_i(r - c_i); reads are gathered, writes aligned and
//                 non-temporal.
//   k_near_nodes, k_chain_wg, k_spread
//                 the same coupling stage for chains of 257..1024 beads: node
//                 velocities around each bead, all substeps in one
//                 1024-thread workgroup writing per-substep records, and the
//                 records turned into node impulses
//   k_fixup       re-collides the nodes the beads touched, with their
//                 impulse, and overwrites their outputs
//   k_collide_deferred, k_overflow
//                 batched steps with chains of 257..1024 beads in sparse
//                 boxes: the tiles holding the beads' node tables skip the
//                 plain collide and are collided with their impulses beside
//                 it, after the coupling; nodes outside them that got an
//                 impulse are fixed up after the collide
//   k_node_field, k_collide_forced
//                 boxes whose beads cover much of the box: node velocities
//                 once per step for the beads' tables, and a collide after
//                 the coupling that takes the node impulses itself
//   k_stats*      FP64 conserved sums, mode variances, negative-population
//                 count; k_chain_obs: centre of mass, R_g^2, R_e^2 (Sec. III.A)
#include "lbmd_device.hpp"
#include "lbmd_kernels.hpp"

namespace lbd {

__device__ __forceinline__ uint32_t div_L(uint32_t r, int L, double inv_L, uint32_t* rem)
{
    uint32_t q = (uint32_t)((double)r * inv_L);
    int32_t rr = (int32_t)(r - q * (uint32_t)L);
    if (rr < 0) { q -= 1; rr += L; }
    else if (rr >= L) { q += 1; rr -= L; }
    *rem = (uint32_t)rr;
    return q;
}

// Index of the node r - c_i for every direction i (periodic), from the node's
// coordinates: the source of the population that arrives at r.
struct Upwind {
    uint32_t X[3], Y[3], Z[3];
    __device__ __forceinline__ Upwind(uint32_t x, uint32_t y, uint32_t z, uint32_t L)
    {
        const uint32_t LL = L * L;
        X[0] = x + 1 == L ? 0 : x + 1; X[1] = x; X[2] = x == 0 ? L - 1 : x - 1;
        Y[0] = (y + 1 == L ? 0 : y + 1) * L; Y[1] = y * L; Y[2] = (y == 0 ? L - 1 : y - 1) * L;
        Z[0] = (z + 1 == L ? 0 : z + 1) * LL; Z[1] = z * LL; Z[2] = (z == 0 ? L - 1 : z - 1) * LL;
    }
    // slot 0 holds coordinate + 1, slot 2 coordinate - 1: r - c_i uses slot c_i + 1
    __device__ __forceinline__ uint32_t src(int i) const { return X[cxv(i) + 1] + Y[cyv(i) + 1] + Z[czv(i) + 1]; }
};

template <typename R, bool NT>
__device__ __forceinline__ void gather_pre(const R* __restrict__ a, const Upwind& up, R d[19])
{
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const uint64_t q = pop_at(i, up.src(i));
        d[i] = NT ? __builtin_nontemporal_load(a + q) : a[q];
    }
}

__device__ __forceinline__ Upwind upwind_of(uint32_t r, int L, double inv_L)
{
    uint32_t x, y;
    const uint32_t q = div_L(r, L, inv_L, &x);
    const uint32_t z = div_L(q, L, inv_L, &y);
    return Upwind(x, y, z, (uint32_t)L);
}

// deferral segment of node `node` of box bx (its stamps sit at 2 * segment
// and 2 * segment + 1)
__device__ __forceinline__ uint32_t dseg_of(const BoxDev& bx, uint32_t node)
{
    return DSEG_PER_TILE * bx.tile_begin + node / DSEG;
}

// -------------------------------------------------------------- collide
// One tile of 256 nodes: gather the pre-collision populations (pull), collide
// with no impulse, write post-collision values aligned and non-temporal.
template <typename R>
__device__ __forceinline__ void collide_tile(const BoxDev* __restrict__ boxes, const CollideConst<R>* __restrict__ ccs,
                                             const uint32_t* __restrict__ tile_box, int fixed_box, uint32_t tile,
                                             const R* __restrict__ A, R* __restrict__ B, Ctrl* __restrict__ ctrl,
                                             uint32_t t, const uint32_t* __restrict__ defer, uint32_t lane)
{
    int bi;
    if (defer) {   // batched steps (every tile's box from tile_box)
        // a deferred segment (this wavefront's nodes) is collided after the
        // coupling, with its impulses (k_collide_deferred); the stamp load
        // goes out beside the box load
        const uint32_t w = __builtin_amdgcn_readfirstlane(lane / DSEG);   // wavefront-uniform: a scalar load
        const uint32_t st = defer[2u * (DSEG_PER_TILE * tile + w) + (t & 1u)];
        bi = (int)tile_box[tile];
        if (st == defer_stamp(t)) return;
    } else {
        bi = fixed_box >= 0 ? fixed_box : (int)tile_box[tile];
    }
    const BoxDev& bx = boxes[bi];
    const int L = bx.L;
    const uint32_t V = (uint32_t)L * L * L;
    const uint32_t r = (tile - bx.tile_begin) * 256u + lane;
    if (r >= V) return;
    const CollideConst<R> cc = ccs[bi];
    const Upwind up = upwind_of(r, L, bx.inv_L);
    R d[19];
    gather_pre<R, false>(A + bx.pop_off, up, d);
    R o[19];
    const uint32_t h = collide<R>(d, o, (R)0, (R)0, (R)0, cc, r, t, bx.seed, bx.box_id);
    R* b = B + bx.pop_off;
#pragma unroll
    for (int i = 0; i < 19; ++i) __builtin_nontemporal_store(o[i], b + pop_at(i, r));
    if (h) atomicOr(&ctrl->health, h);
}

// Launch shapes the autotuner chooses from: W caps the waves per SIMD (4..8);
// BT threads per block collide BT / 256 consecutive 256-node tiles (256, 512
// or 1024 nodes per block); PERSIST selects a grid of a few blocks per CU
// that strides over the tiles instead of one block per tile group.  Every
// node gets the same per-node arithmetic, so all shapes compute the same bits.
template <typename R, int W, bool PERSIST, int BT = 256>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(1, W))) void k_collide(
    const BoxDev* __restrict__ boxes, const CollideConst<R>* __restrict__ ccs, const uint32_t* __restrict__ tile_box,
    int fixed_box, uint32_t tile0, uint32_t n_tiles, const R* __restrict__ A, R* __restrict__ B,
    Ctrl* __restrict__ ctrl, uint32_t s_off, const uint32_t* __restrict__ defer)
{
    constexpr uint32_t M = BT / 256;   // 256-node tiles per block
    const uint32_t t = ctrl->step + s_off;
    if constexpr (M == 1) {
        if (PERSIST) {
            for (uint32_t k = blockIdx.x; k < n_tiles; k += gridDim.x)
                collide_tile<R>(boxes, ccs, tile_box, fixed_box, tile0 + k, A, B, ctrl, t, defer, threadIdx.x);
        } else {
            collide_tile<R>(boxes, ccs, tile_box, fixed_box, tile0 + blockIdx.x, A, B, ctrl, t, defer, threadIdx.x);
        }
    } else {
        const uint32_t sub = threadIdx.x / 256u, lane = threadIdx.x % 256u;
        if (PERSIST) {
            for (uint32_t k = blockIdx.x * M + sub; k < n_tiles; k += gridDim.x * M)
                collide_tile<R>(boxes, ccs, tile_box, fixed_box, tile0 + k, A, B, ctrl, t, defer, lane);
        } else {
            const uint32_t k = blockIdx.x * M + sub;
            if (k < n_tiles) collide_tile<R>(boxes, ccs, tile_box, fixed_box, tile0 + k, A, B, ctrl, t, defer, lane);
        }
    }
}

// --------------------------------------------------------------- couple
struct ChainArgs {
    double* x; double* v; double* f; double* fc;   // [total beads][3]
    int32_t* nl_cnt; uint16_t* nl_idx; double* nl_x0; int nl_cap;
    unsigned long long* imp;   // dense impulse field, 3 per node (global node index), fixed point
    uint32_t* touched;         // per bead: local nodes it handed impulse to this step
    int32_t* touched_cnt;
    int touch_cap;             // slots per bead: 8 x (substeps + 1), one stencil change per substep at most
    uint32_t* nl_rebuilds;     // per box: neighbour-list builds so far (diagnostic)
    double* vhist; int hist_len; uint64_t total_beads;
    double* tape;              // non-null while replaying a window segment: per substep and bead,
                               // TAPE_REC doubles (see k_couple)
    double* tape_x0;           // with tape: the step's starting x, v (at tape_vo), f (at tape_fo)
    uint64_t tape_vo, tape_fo;
    uint32_t* defer;           // non-null when the step defers tiles: per collide tile, the stamp of
                               // the last step that deferred it
    uint32_t* dclaim;          // per collide tile: stamp of the last step that listed it
    uint32_t* defer_list; uint32_t defer_cap;
    uint32_t* ovf; uint32_t ovf_cap;   // (bead, local node) pairs outside the deferred tiles
    uint32_t* ovm;             // per global node: stamp of the last step that listed it in ovf
};

// node velocities (MD units) of the 8 stencil nodes from the frozen populations;
// the loads of NB nodes are issued before any of them is used (NB = 8: one
// round trip to memory, for register-rich callers)
template <typename R, typename U, int NB>
__device__ __forceinline__ void stencil_velocities(const R* __restrict__ a, const int i0[3], int L,
                                                   double rho0, double inv_tau, U u[8][3])
{
    static_assert(NB == 1 || NB == 2 || NB == 4 || NB == 8, "NB divides 8");
#pragma unroll
    for (int k0 = 0; k0 < 8; k0 += NB) {
        R d[NB][19];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const int kk = k0 + k;
            const int ix = i0[0] + (kk & 1), iy = i0[1] + ((kk >> 1) & 1), iz = i0[2] + ((kk >> 2) & 1);
            const Upwind up((uint32_t)(ix >= L ? ix - L : ix), (uint32_t)(iy >= L ? iy - L : iy),
                            (uint32_t)(iz >= L ? iz - L : iz), (uint32_t)L);
            gather_pre<R, false>(a, up, d[k]);
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
            for (int i = 0; i < 19; ++i) {
                const double di = (double)d[k][i];
                rho += di;
                if (cxv(i)) jx += cxv(i) * di;
                if (cyv(i)) jy += cyv(i) * di;
                if (czv(i)) jz += czv(i) * di;
            }
            rho += rho0;
            u[k0 + k][0] = (U)(jx / rho * inv_tau);
            u[k0 + k][1] = (U)(jy / rho * inv_tau);
            u[k0 + k][2] = (U)(jz / rho * inv_tau);
        }
    }
}

// stencil_velocities over the T lanes of one bead (T = 8 / NK, or 16 with the
// upper eight lanes repeating the lower): lane l gathers corners l, l + T8,
// ... (NK of them, T8 = 8 / NK), and the lanes then exchange them, so that
// every lane ends with all eight corners, computed as stencil_velocities
// computes them
template <typename R, int NK>
__device__ __forceinline__ void stencil_shared(const R* __restrict__ a, const int i0[3], int L, double rho0,
                                               double inv_tau, int lane, int T, R u[8][3])
{
    constexpr int T8 = 8 / NK;
    R d[NK][19];
    const int k0 = lane & (T8 - 1);
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const int kk = k0 + k * T8;
        const int ix = i0[0] + (kk & 1), iy = i0[1] + ((kk >> 1) & 1), iz = i0[2] + ((kk >> 2) & 1);
        const Upwind up((uint32_t)(ix >= L ? ix - L : ix), (uint32_t)(iy >= L ? iy - L : iy),
                        (uint32_t)(iz >= L ? iz - L : iz), (uint32_t)L);
        gather_pre<R, false>(a, up, d[k]);
    }
    R own[NK][3];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const double di = (double)d[k][i];
            rho += di;
            if (cxv(i)) jx += cxv(i) * di;
            if (cyv(i)) jy += cyv(i) * di;
            if (czv(i)) jz += czv(i) * di;
        }
        rho += rho0;
        own[k][0] = (R)(jx / rho * inv_tau);
        own[k][1] = (R)(jy / rho * inv_tau);
        own[k][2] = (R)(jz / rho * inv_tau);
    }
    // corner k sits in slot k / T8 of lane k % T8 of the bead's lanes
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) u[k][c] = __shfl(own[k / T8][c], k % T8, T);
}

constexpr int MAXB = 1024;
constexpr double NL_SKIN = 0.5;

// first and last bead of bead b's chain: a box's beads form chains of
// chain_len consecutive indices (one chain, or the several chains of a
// semidilute solution, Sec. III.C)
struct ChainSpan { int lo, hi; };
__device__ __forceinline__ ChainSpan chain_span(const BoxDev& bx, int b)
{
    const int n = bx.chain_len;
    const int lo = b - b % n;
    return ChainSpan{lo, lo + n - 1};
}

// FENE force on bead b from its bonded neighbours, b - 1 and b + 1 when they
// are on its chain (Sec. II.A), unwrapped separations
__device__ __forceinline__ uint32_t fene_force(const BoxDev& bx, int b, ChainSpan sp, const double x[3],
                                               const double* xs, double F[3])
{
    uint32_t hb = 0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int j = side ? b + 1 : b - 1;
        if (j < sp.lo || j > sp.hi) continue;
        const double d0 = x[0] - xs[3 * j], d1 = x[1] - xs[3 * j + 1], d2 = x[2] - xs[3 * j + 2];
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        double den = 1.0 - r2 * bx.inv_r0sq;
        if (!(den > 0.0)) { hb |= H_FENE; den = 1e-12; }
        const double gf = -bx.k_fene / den;
        F[0] += gf * d0; F[1] += gf * d1; F[2] += gf * d2;
    }
    return hb;
}

// purely repulsive LJ on bead b from beads j0, j0+T, j0+2T, j0+3T (those < N
// and != b): the four separations are independent, so their latencies overlap;
// the forces are added in ascending j.
template <typename IDX>
__device__ __forceinline__ void wca_add4(const double x[3], const double* xs, IDX jof, int k0, int kend, int step,
                                         int b, double Ld, double iL, double rc2, double sigsq, double eps24,
                                         double F[3])
{
    double d[4][3], r2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = k0 + u * step;
        const int j = k < kend ? jof(k) : b;
        d[u][0] = x[0] - xs[3 * j]; d[u][1] = x[1] - xs[3 * j + 1]; d[u][2] = x[2] - xs[3 * j + 2];
        d[u][0] -= Ld * rint(d[u][0] * iL); d[u][1] -= Ld * rint(d[u][1] * iL); d[u][2] -= Ld * rint(d[u][2] * iL);
        r2[u] = j == b ? rc2 : d[u][0] * d[u][0] + d[u][1] * d[u][1] + d[u][2] * d[u][2];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (r2[u] < rc2) {
            const double ir2 = 1.0 / r2[u];
            const double s2 = sigsq * ir2;
            const double s6 = s2 * s2 * s2;
            const double gf = eps24 * s6 * (2.0 * s6 - 1.0) * ir2;
            F[0] += gf * d[u][0]; F[1] += gf * d[u][1]; F[2] += gf * d[u][2];
        }
    }
}

// purely repulsive LJ on bead b from bead j (minimum image), cut at 2^(1/6) sigma
__device__ __forceinline__ void wca_add(const double x[3], const double* xs, int j, double Ld, double iL,
                                        double rc2, double sigsq, double eps24, double F[3])
{
    double d0 = x[0] - xs[3 * j], d1 = x[1] - xs[3 * j + 1], d2 = x[2] - xs[3 * j + 2];
    d0 -= Ld * rint(d0 * iL); d1 -= Ld * rint(d1 * iL); d2 -= Ld * rint(d2 * iL);
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    if (r2 < rc2) {
        const double ir2 = 1.0 / r2;
        const double s2 = sigsq * ir2;
        const double s6 = s2 * s2 * s2;
        const double gf = eps24 * s6 * (2.0 * s6 - 1.0) * ir2;
        F[0] += gf * d0; F[1] += gf * d1; F[2] += gf * d2;
    }
}

// initial last-force of every bead: the conservative force at the start positions
__global__ __launch_bounds__(1024) void k_init_forces(const BoxDev* __restrict__ boxes,
                                                      const int32_t* __restrict__ couple_list,
                                                      double* __restrict__ xg, double* __restrict__ fg,
                                                      Ctrl* __restrict__ ctrl)
{
    __shared__ double xs[3 * MAXB];
    const BoxDev& bx = boxes[couple_list[blockIdx.x]];
    const int N = bx.N, b = threadIdx.x;
    const uint64_t g = bx.bead_off + b;
    double x[3] = {0, 0, 0};
    if (b < N)
        for (int c = 0; c < 3; ++c) { x[c] = xg[3 * g + c]; xs[3 * b + c] = x[c]; }
    __syncthreads();
    if (b < N) {
        double F[3] = {0, 0, 0};
        uint32_t hb = fene_force(bx, b, chain_span(bx, b), x, xs, F);
        double W[3] = {0, 0, 0};
        for (int j = 0; j < N; ++j)
            if (j != b) wca_add(x, xs, j, (double)bx.L, bx.inv_L, bx.rc2, bx.sigsq, 24.0 * bx.eps, W);
        for (int c = 0; c < 3; ++c) fg[3 * g + c] = F[c] + W[c];
        if (hb) atomicOr(&ctrl->health, hb);
    }
}

// hand one stencil's accumulated impulse (MD units) to the dense field and
// list the nodes; no result is waited on
__device__ __forceinline__ uint32_t flush_stencil(const ChainArgs& ca, uint64_t node_off, uint64_t g,
                                                  const uint32_t cnode[8], double acc[8][3], double tau,
                                                  int& tcnt)
{
    uint32_t hb = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        unsigned long long* dst = ca.imp + 3 * (node_off + cnode[k]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double v = acc[k][c] * tau;      // lattice momentum units
            if (!(fabs(v) < IMP_MAX)) { hb |= H_FIXED; v = 0.0; }
            atomicAdd(dst + c, (unsigned long long)(long long)llrint(v * IMP_SCALE));
        }
        if (tcnt < ca.touch_cap) ca.touched[g * ca.touch_cap + tcnt] = cnode[k];
        else hb |= H_TABLE;
        ++tcnt;
    }
    return hb;
}

// One workgroup per chain; T lanes per bead split the pair loop.  Threads
// 0..T*Npad-1: bead b = tid / T, lane = tid % T.  All T lanes of a bead
// compute the same bead update (their force partial sums are combined by a
// butterfly, which gives every lane the same bits); lane 0 writes.
// Lane l of bead b owns the partners j = l, l + T, l + 2T, ... (j != b).  It
// keeps the ones within the list radius (cut-off plus NL_SKIN) in its own
// list, in ascending j, built at the first substep and again whenever some
// bead of the chain has moved more than half the skin since the last build:
// every partner within the cut-off is then on the list, and the list holds
// them in the order of the full scan, so the forces are the same bits.  A
// lane whose partners within the list radius exceed its slots scans all of
// them instead.
constexpr int CPL_SLOTS = 32;   // list slots per lane of the one-workgroup coupling kernel
template <typename R, int MAXT = 256>
__global__ __launch_bounds__(MAXT) void k_couple(const BoxDev* __restrict__ boxes,
                                                 const int32_t* __restrict__ couple_list,
                                                 const R* __restrict__ A, ChainArgs ca,
                                                 Ctrl* __restrict__ ctrl, uint32_t s_off)
{
    __shared__ double xs[3 * BIG_CHAIN];   // chains on this path have at most BIG_CHAIN beads
    static_assert(BIG_CHAIN <= 256, "partner indices are stored in one byte");
    __shared__ uint8_t nl[MAXT * CPL_SLOTS + 4];   // per lane: its partners within the list radius
    __shared__ int moved[2];                        // per substep parity: a bead moved past half the skin
    __builtin_amdgcn_s_setprio(3);   // latency-bound chain beside the bandwidth-bound collide
    const int bi = couple_list[blockIdx.x];
    const BoxDev bx = boxes[bi];   // a copy: its fields stay in registers across the substeps
    const int N = bx.N;
    // lanes per bead depend on this chain's length alone, so a box computes
    // the same bits in any batch
    const int T = bx.couple_T;
    const int b = threadIdx.x / T, lane = threadIdx.x % T;
    const bool act = b < N;
    const bool writer = act && lane == 0;
    const uint64_t g = bx.bead_off + (uint64_t)(act ? b : 0);
    const ChainSpan sp = chain_span(bx, act ? b : 0);
    const uint32_t t = ctrl->step + s_off;
    const int L = bx.L;
    const double Ld = (double)L, iL = bx.inv_L;
    const double dt = bx.dt, hdt_m = 0.5 * dt / bx.mass;
    const double inv_tau = 1.0 / bx.tau_lb;
    const double eps24 = 24.0 * bx.eps;
    const R* a = A + bx.pop_off;
    // list radius, a hair above cut-off plus skin so that rounding cannot
    // drop a partner that comes within the cut-off
    const double rl = sqrt(bx.rc2) + NL_SKIN + 1e-6;
    const double rl2 = rl * rl;
    const uint32_t nl_base = threadIdx.x * CPL_SLOTS;
    if (threadIdx.x == 0) { moved[0] = 0; moved[1] = 0; }

    double x[3] = {0, 0, 0}, v[3] = {0, 0, 0}, f[3] = {0, 0, 0}, fcl[3] = {0, 0, 0};
    if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) { x[c] = ca.x[3 * g + c]; v[c] = ca.v[3 * g + c]; f[c] = ca.f[3 * g + c]; }
        if (ca.tape_x0 && lane == 0)   // the step's starting beads, for the adjoint
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                ca.tape_x0[3 * g + c] = x[c];
                ca.tape_x0[ca.tape_vo + 3 * g + c] = v[c];
                ca.tape_x0[ca.tape_fo + 3 * g + c] = f[c];
            }
    }
    int cb[3] = {-1, -1, -1};     // base cell of the cached stencil
    // node velocities of the cached stencil (MD units), kept in the storage
    // precision: FP32 storage carries no more digits than that
    R cu[8][3];
    double acc[8][3];             // impulse accumulated on the cached stencil (MD units)
    uint32_t cnode[8];
    bool have_acc = false;
    uint32_t hbits = 0;
    int tcnt = 0;
    double x0[3] = {0, 0, 0};     // position at the last list build
    int nl_n = -1;                // entries of this lane's list (-1: the lane scans all its partners)

    for (int s = 0; s < bx.substeps; ++s) {
        if (act) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v[c] += f[c] * hdt_m;
                x[c] += v[c] * dt;
            }
            if (lane == 0) {
                xs[3 * b] = x[0]; xs[3 * b + 1] = x[1]; xs[3 * b + 2] = x[2];
                const double e0 = x[0] - x0[0], e1 = x[1] - x0[1], e2 = x[2] - x0[2];
                if (s > 0 && e0 * e0 + e1 * e1 + e2 * e2 > 0.25 * NL_SKIN * NL_SKIN) moved[s & 1] = 1;
            }
        }
        __syncthreads();
        // the same for every thread: the flag of this parity was cleared a
        // substep ago, and the other parity's is cleared now, after every
        // read of it
        const bool rebuild = s == 0 || moved[s & 1] != 0;
        if (threadIdx.x == 0) moved[(s + 1) & 1] = 0;
        if (act) {
            if (rebuild) {
                x0[0] = x[0]; x0[1] = x[1]; x0[2] = x[2];
                int cnt = 0;
                for (int j = lane; j < N; j += T) {
                    double d0 = x[0] - xs[3 * j], d1 = x[1] - xs[3 * j + 1], d2 = x[2] - xs[3 * j + 2];
                    d0 -= Ld * rint(d0 * iL); d1 -= Ld * rint(d1 * iL); d2 -= Ld * rint(d2 * iL);
                    if (j != b && d0 * d0 + d1 * d1 + d2 * d2 < rl2) {
                        if (cnt < CPL_SLOTS) nl[nl_base + cnt] = (uint8_t)j;
                        ++cnt;
                    }
                }
                nl_n = cnt <= CPL_SLOTS ? cnt : -1;
            }
            // repulsive LJ over this lane's share of the partners
            double W[3] = {0, 0, 0};
            if (nl_n >= 0) {
                auto jl = [&](int k) { return (int)nl[nl_base + k]; };
                for (int k = 0; k < nl_n; k += 4) wca_add4(x, xs, jl, k, nl_n, 1, b, Ld, iL, bx.rc2, bx.sigsq, eps24, W);
            } else {
                auto jof = [](int k) { return k; };
                for (int j = lane; j < N; j += 4 * T) wca_add4(x, xs, jof, j, N, T, b, Ld, iL, bx.rc2, bx.sigsq, eps24, W);
            }
            for (int o = 1; o < T; o <<= 1) {
#pragma unroll
                for (int c = 0; c < 3; ++c) W[c] += __shfl_xor(W[c], o, T);
            }
            double F[3] = {0, 0, 0};
            hbits |= fene_force(bx, b, sp, x, xs, F);
            F[0] += W[0]; F[1] += W[1]; F[2] += W[2];
            // stencil of the bead: nodes at integer coordinates, periodic
            int i0[3];
            double fr[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double xt = x[c] - Ld * floor(x[c] * iL);
                const double fl = floor(xt);
                fr[c] = xt - fl;
                int ii = (int)fl;
                if (ii >= L) ii -= L;
                if (ii < 0) ii += L;
                i0[c] = ii;
            }
            if (i0[0] != cb[0] || i0[1] != cb[1] || i0[2] != cb[2]) {
                if (have_acc && lane == 0) hbits |= flush_stencil(ca, bx.node_off, g, cnode, acc, bx.tau_lb, tcnt);
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int ix = i0[0] + (k & 1), iy = i0[1] + ((k >> 1) & 1), iz = i0[2] + ((k >> 2) & 1);
                    cnode[k] = (uint32_t)(ix >= L ? ix - L : ix) +
                               (uint32_t)L * ((uint32_t)(iy >= L ? iy - L : iy) + (uint32_t)L * (uint32_t)(iz >= L ? iz - L : iz));
                    acc[k][0] = acc[k][1] = acc[k][2] = 0.0;
                }
                // the bead's lanes share the gathers (T is uniform over the workgroup)
                if (T >= 8) stencil_shared<R, 1>(a, i0, L, bx.rho0, inv_tau, lane, T, cu);
                else if (T == 4) stencil_shared<R, 2>(a, i0, L, bx.rho0, inv_tau, lane, T, cu);
                else if (T == 2) stencil_shared<R, 4>(a, i0, L, bx.rho0, inv_tau, lane, T, cu);
                else stencil_velocities<R, R, 8>(a, i0, L, bx.rho0, inv_tau, cu);
                cb[0] = i0[0]; cb[1] = i0[1]; cb[2] = i0[2];
                have_acc = true;
            }
            double wt[8], ub[3] = {0, 0, 0};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                wt[k] = ((k & 1) ? fr[0] : 1.0 - fr[0]) * (((k >> 1) & 1) ? fr[1] : 1.0 - fr[1]) *
                        (((k >> 2) & 1) ? fr[2] : 1.0 - fr[2]);
                ub[0] += wt[k] * (double)cu[k][0]; ub[1] += wt[k] * (double)cu[k][1]; ub[2] += wt[k] * (double)cu[k][2];
            }
            const U4 w = philox10(U4{(uint32_t)b, t, (1u << 16) | (uint32_t)s, 0u}, bx.seed, bx.box_id);
            const uint32_t ws[3] = {w.x, w.y, w.z};
            double* tp = (ca.tape && lane == 0) ? ca.tape + ((uint64_t)s * ca.total_beads + g) * TAPE_REC : nullptr;
            if (tp) {   // substep record for the adjoint: x1, v1, fc, base cell, fractions, node velocities
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    tp[c] = x[c]; tp[3 + c] = v[c]; tp[9 + c] = (double)i0[c]; tp[12 + c] = fr[c];
                }
#pragma unroll
                for (int k = 0; k < 8; ++k)
#pragma unroll
                    for (int c = 0; c < 3; ++c) tp[15 + 3 * k + c] = (double)cu[k][c];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double ffr = -bx.zeta * (v[c] - ub[c]);
                const double frn = bx.bead_noise * unit_noise<double>(ws[c]);
                fcl[c] = ffr + frn;
                f[c] = F[c] + fcl[c];
                v[c] += f[c] * hdt_m;
            }
            if (tp) { tp[6] = fcl[0]; tp[7] = fcl[1]; tp[8] = fcl[2]; }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                acc[k][0] -= wt[k] * fcl[0] * dt;
                acc[k][1] -= wt[k] * fcl[1] * dt;
                acc[k][2] -= wt[k] * fcl[2] * dt;
            }
        }
        __syncthreads();
    }
    if (writer) {
        if (have_acc) hbits |= flush_stencil(ca, bx.node_off, g, cnode, acc, bx.tau_lb, tcnt);
        ca.touched_cnt[g] = tcnt < ca.touch_cap ? tcnt : ca.touch_cap;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ca.x[3 * g + c] = x[c]; ca.v[3 * g + c] = v[c]; ca.f[3 * g + c] = f[c]; ca.fc[3 * g + c] = fcl[c];
        }
        if (ca.vhist) {
            double* hv = ca.vhist + ((uint64_t)(t % (uint32_t)ca.hist_len) * ca.total_beads + g) * 3;
            hv[0] = v[0]; hv[1] = v[1]; hv[2] = v[2];
        }
    }
    if (act && hbits) atomicOr(&ctrl->health, hbits);
}

// ------------------------------------------------- couple, large chains
// Chains above 256 beads take three launches per LB step, on one stream:
//   k_near_nodes  every bead's 3x3x3 nodes around its nearest node: the node
//                 velocities (MD units), one thread per (bead, node), so all
//                 the population loads of the stage go out in one wave;
//   k_chain_wg    one workgroup of up to 1024 threads per box, one thread
//                 per bead, every MD substep in one launch.  Positions,
//                 neighbour lists, the positions they were built at and the
//                 cell buckets of the list build live in LDS (150 KB); each
//                 bead's stencil velocities in
//                 registers, refilled from the 3x3x3 table when the bead
//                 changes cell.  Per substep each bead writes one record
//                 (fractions, coupling force, base cell) instead of handing
//                 impulses over, so no atomic traffic sits in the barrier-
//                 synchronised substep loop;
//   k_spread      one thread per (bead, stencil corner) turns the records into
//                 node impulses: the same accumulation per stencil as the
//                 one-workgroup path of small chains, then one fixed-point
//                 atomic per component and stencil.
constexpr int WG_MAXB = 1024;
constexpr int NEAR = 27;    // nodes in the table of one bead

// Neighbour-list build over cells: nc cells per axis, each at least the list
// radius wide (plus a margin far above rounding), so every partner within the
// radius lies in the 3x3x3 cells around a bead's own.  A cell's bucket is its
// coordinates mod 16 (4096 buckets): the 27 cells around any cell land in 27
// distinct buckets when nc <= 16, or when nc mod 16 is neither 1 nor 2, which
// list_cells ensures (it keeps nc mod 8 off 1 and 2 above 8 by taking fewer,
// wider cells).  Beads of other cells that share a bucket fail the distance
// test.  The test runs in FP32 on positions wrapped into the box, against a
// radius 1e-3 above the list radius: an FP32 rounding of the coordinates
// (under 2.5e-4 for L <= 1625) cannot drop a partner, and the few extra
// partners are skipped by the force loop's exact cut-off test.
constexpr int NBK = 4096;
constexpr double NL_FP32_MARGIN = 1e-3;
__device__ __forceinline__ int list_cells(int L, double rl)
{
    int nc = (int)floor((double)L / (rl + 1e-6));
    if (nc > 8 && (nc % 8 == 1 || nc % 8 == 2)) nc -= nc % 8;
    return nc;
}
__device__ __forceinline__ int wrap_cell(int q, int nc) { return q < 0 ? q + nc : (q >= nc ? q - nc : q); }
__device__ __forceinline__ int bucket_of(int cx, int cy, int cz) { return (cx & 15) | ((cy & 15) << 4) | ((cz & 15) << 8); }

// base-cell index and fraction of one coordinate (periodic, nodes at integers)
__device__ __forceinline__ int cell_of(double xc, int L, double Ld, double iL, double& fr)
{
    const double xt = xc - Ld * floor(xc * iL);
    const double fl = floor(xt);
    fr = xt - fl;
    int ii = (int)fl;
    if (ii >= L) ii -= L;
    if (ii < 0) ii += L;
    return ii;
}

__device__ __forceinline__ uint32_t node_of(int ix, int iy, int iz, int L)
{
    ix = ix >= L ? ix - L : (ix < 0 ? ix + L : ix);
    iy = iy >= L ? iy - L : (iy < 0 ? iy + L : iy);
    iz = iz >= L ? iz - L : (iz < 0 ? iz + L : iz);
    return (uint32_t)ix + (uint32_t)L * ((uint32_t)iy + (uint32_t)L * (uint32_t)iz);
}

// nearest node of a bead position, per axis
__device__ __forceinline__ int nearest_of(double xc, int L, double Ld, double iL)
{
    const double xt = xc - Ld * floor(xc * iL);
    int n = (int)floor(xt + 0.5);
    return n >= L ? n - L : n;
}

// fluid velocity of one node in MD units (u = j / rho / tau_lb) from its
// gathered pre-collision deviations
template <typename R>
__device__ __forceinline__ void node_velocity(const R d[19], double rho0, double inv_tau, R u[3])
{
    double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const double di = (double)d[i];
        rho += di;
        if (cxv(i)) jx += cxv(i) * di;
        if (cyv(i)) jy += cyv(i) * di;
        if (czv(i)) jz += czv(i) * di;
    }
    rho += rho0;
    u[0] = (R)(jx / rho * inv_tau);
    u[1] = (R)(jy / rho * inv_tau);
    u[2] = (R)(jz / rho * inv_tau);
}

// dense boxes: the velocity of every node, once per LB step, so that their
// beads' tables read 3 values per node instead of gathering 19 populations
// (the tables of a dense box cover it several times over)
template <typename R>
__global__ __launch_bounds__(256) void k_node_field(const BoxDev* __restrict__ boxes,
                                                    const int32_t* __restrict__ list, const R* __restrict__ A,
                                                    R* __restrict__ field)
{
    const BoxDev& bx = boxes[list[blockIdx.y]];
    if (!bx.dense) return;
    const int L = bx.L;
    const uint32_t V = (uint32_t)L * L * L;
    const uint32_t r = blockIdx.x * 256u + threadIdx.x;
    if (r >= V) return;
    const Upwind up = upwind_of(r, L, bx.inv_L);
    R d[19];
    gather_pre<R, false>(A + bx.pop_off, up, d);
    R u[3];
    node_velocity<R>(d, bx.rho0, 1.0 / bx.tau_lb, u);
    R* o = field + 3 * (bx.field_off + r);
    o[0] = u[0]; o[1] = u[1]; o[2] = u[2];
}

// the box fields a fix-up uses, read once
struct FixBox {
    int L;
    uint32_t seed, box_id;
    uint64_t pop_off, node_off;
    double inv_L;
};
__device__ __forceinline__ FixBox fix_box(const BoxDev& bx)
{
    return FixBox{bx.L, bx.seed, bx.box_id, bx.pop_off, bx.node_off, bx.inv_L};
}

// fix-up of one node after the plain collide: defined with the fix-up kernels
template <typename R>
__device__ __forceinline__ void fixup_node(const FixBox& bx, const CollideConst<R>& cc, uint32_t r,
                                           unsigned long long* __restrict__ imp, uint32_t* __restrict__ claim,
                                           const R* __restrict__ A, R* __restrict__ B, Ctrl* __restrict__ ctrl,
                                           uint32_t t, int keep_imp);

// the same fix-up (impulses left in the field), the node claimed before its
// populations are read: fewer live registers, for a rare path inside a
// bandwidth-bound kernel
template <typename R>
__device__ __forceinline__ void fixup_node_claim_first(const BoxDev& bx, const CollideConst<R>* __restrict__ ccs,
                                                       int bi, uint32_t r, const unsigned long long* __restrict__ imp,
                                                       uint32_t* __restrict__ claim, const R* __restrict__ A,
                                                       R* __restrict__ B, Ctrl* __restrict__ ctrl, uint32_t t)
{
    const uint64_t node = bx.node_off + r;
    if (atomicExch(&claim[node], t + 1u) == t + 1u) return;   // another caller took this node
    R d[19];
    gather_pre<R, false>(A + bx.pop_off, upwind_of(r, bx.L, bx.inv_L), d);
    const unsigned long long* q = imp + 3 * node;
    const R fx = (R)((double)(long long)q[0] * IMP_INV_SCALE), fy = (R)((double)(long long)q[1] * IMP_INV_SCALE),
            fz = (R)((double)(long long)q[2] * IMP_INV_SCALE);
    R o[19];
    const uint32_t h = collide<R>(d, o, fx, fy, fz, ccs[bi], r, t, bx.seed, bx.box_id);
    R* b = B + bx.pop_off;
#pragma unroll
    for (int i = 0; i < 19; ++i) b[pop_at(i, r)] = o[i];
    if (h) atomicOr(&ctrl->health, h);
}

// The node table of the step, one (bead, table node) item per thread: item
// `item` of list entry `li`.  With Aprev (batched steps that defer tiles,
// from the second step of a run of steps on) it also finishes the previous
// step first: the impulses that landed outside that step's deferred tiles are
// collided again (Aprev -> A, the previous step's number), their impulses
// left in the field for the chain kernel to clear; this thread takes entries
// fix_e0, fix_e0 + fix_n, ...  A table node whose population comes from such
// a node takes the fixed value computed here instead of reading it, so no
// thread reads what another writes.  With `stamp` the item also stamps its
// node's collide tile as deferred in step t.
template <typename R>
__device__ __forceinline__ void near_work(const BoxDev* __restrict__ boxes, const int32_t* __restrict__ list,
                                          R* A, const ChainArgs& ca, R* __restrict__ near_u,
                                          int4* __restrict__ near_c, const R* __restrict__ field, Ctrl* ctrl,
                                          uint32_t t, const CollideConst<R>* __restrict__ ccs,
                                          const int32_t* __restrict__ bead_box, uint32_t* __restrict__ claim,
                                          const R* __restrict__ Aprev, int one_box, const BoxDev& one, int li,
                                          int item, uint32_t fix_e0, uint32_t fix_n, bool stamp)
{
    uint32_t n_pend = 0;
    if (Aprev) {
        n_pend = min(ctrl->ovf_cnt, ca.ovf_cap);
        for (uint32_t e = fix_e0; e < n_pend; e += fix_n) {
            const uint64_t g = ca.ovf[2 * (uint64_t)e];
            const uint32_t r = ca.ovf[2 * (uint64_t)e + 1];
            const int bi = bead_box[g];
            fixup_node<R>(fix_box(boxes[bi]), ccs[bi], r, ca.imp, claim, Aprev, A, ctrl, t - 1u, 1);
        }
    }
    // one_box >= 0: the launch covers that box alone, its descriptor passed by
    // value (no dependent loads of the box list and table before the beads')
    const int bi = one_box >= 0 ? one_box : list[li];
    const BoxDev bx = one_box >= 0 ? one : boxes[bi];   // a copy: its fields stay in registers
    const int N = bx.N, L = bx.L;
    if (item >= N * NEAR) return;
    const int b = item / NEAR, q = item - b * NEAR;
    const uint64_t g = bx.bead_off + (uint64_t)b;
    const double Ld = (double)L, iL = bx.inv_L;
    const int n0 = nearest_of(ca.x[3 * g], L, Ld, iL), n1 = nearest_of(ca.x[3 * g + 1], L, Ld, iL),
              n2 = nearest_of(ca.x[3 * g + 2], L, Ld, iL);
    if (q == 0) near_c[g] = make_int4(n0, n1, n2, 0);
    const int ix = n0 - 1 + q % 3, iy = n1 - 1 + (q / 3) % 3, iz = n2 - 1 + q / 9;
    const uint32_t node = node_of(ix, iy, iz, L);
    R* o = near_u + (g * NEAR + (uint64_t)q) * 3;
    if (bx.dense) {
        const R* fu = field + 3 * (bx.field_off + node);
        o[0] = fu[0]; o[1] = fu[1]; o[2] = fu[2];
        return;
    }
    const uint32_t nz = node / ((uint32_t)L * (uint32_t)L), rem = node - nz * (uint32_t)L * (uint32_t)L;
    const uint32_t ny = rem / (uint32_t)L, nx = rem - ny * (uint32_t)L;
    const Upwind up(nx, ny, nz, (uint32_t)L);
    R d[19];
    gather_pre<R, false>(A + bx.pop_off, up, d);
    if (n_pend) {
        // directions whose source node the previous step listed; every array
        // index below is a compile-time constant, so d and oo stay in registers
        const uint32_t pst = defer_stamp(t - 1u);
        uint32_t need = 0;
#pragma unroll
        for (int i = 0; i < 19; ++i)
            if (ca.ovm[bx.node_off + up.src(i)] == pst) need |= 1u << i;
        while (need) {
            const int ik = __builtin_ctz(need);
            need &= need - 1u;
            uint32_t src = 0;
#pragma unroll
            for (int j = 0; j < 19; ++j)
                if (j == ik) src = up.src(j);
            R dd[19], oo[19];
            gather_pre<R, false>(Aprev + bx.pop_off, upwind_of(src, L, bx.inv_L), dd);
            const unsigned long long* qi = ca.imp + 3 * (bx.node_off + src);
            const R fx = (R)((double)(long long)qi[0] * IMP_INV_SCALE),
                    fy = (R)((double)(long long)qi[1] * IMP_INV_SCALE),
                    fz = (R)((double)(long long)qi[2] * IMP_INV_SCALE);
            (void)collide<R>(dd, oo, fx, fy, fz, ccs[bi], src, t - 1u, bx.seed, bx.box_id);
#pragma unroll
            for (int j = 0; j < 19; ++j)
                if (j == ik) d[j] = oo[j];
        }
    }
    if (stamp && ca.defer)   // the bead's stencil stays on its table's nodes while it moves
                             // less than half a cell from its nearest node: their tiles wait
                             // for the impulses (a plain store: every writer stores the same stamp)
        ca.defer[2u * dseg_of(bx, node) + (t & 1u)] = defer_stamp(t);
    R u[3];
    node_velocity<R>(d, bx.rho0, 1.0 / bx.tau_lb, u);
    o[0] = u[0]; o[1] = u[1]; o[2] = u[2];
}

// The node-table kernel: grid (items of the largest chain / 256, list
// entries).  zero_head: a run of steps starts here; its later collides count
// their node-table workgroups from zero.
template <typename R>
__global__ __launch_bounds__(256) void k_near_nodes(const BoxDev* __restrict__ boxes,
                                                    const int32_t* __restrict__ list, R* A,
                                                    ChainArgs ca, R* __restrict__ near_u, int4* __restrict__ near_c,
                                                    const R* __restrict__ field, Ctrl* __restrict__ ctrl,
                                                    uint32_t s_off, const CollideConst<R>* __restrict__ ccs,
                                                    const int32_t* __restrict__ bead_box,
                                                    uint32_t* __restrict__ claim, const R* __restrict__ Aprev,
                                                    int one_box, BoxDev one, int zero_head)
{
    const uint32_t t = ctrl->step + s_off;
    if (zero_head && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 2) {
        ctrl->head_done[threadIdx.x] = 0u;
        ctrl->head_fix[threadIdx.x] = 0u;
    }
    const uint32_t nth = gridDim.x * gridDim.y * blockDim.x;
    const uint32_t e0 = (blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
    near_work<R>(boxes, list, A, ca, near_u, near_c, field, ctrl, t, ccs, bead_box, claim, Aprev, one_box, one,
                 (int)blockIdx.y, (int)(blockIdx.x * blockDim.x + threadIdx.x), e0, nth, true);
}

// Step t's collide in a run of batched steps that carries its own node
// tables: workgroups 0..n_head-1 do the node-table kernel's work (step t's
// tables; the tiles were stamped by the previous step's chain kernel) and
// count themselves done in head_done[t & 1]; the chain kernel, already
// resident on another queue, waits for that count.  The other workgroups
// collide one tile each, like k_collide.  When the previous step listed
// impulses outside its deferred tiles, the node-table workgroups first fix
// those nodes up and wait for each other (head_fix), so that the tables read
// the fixed values; and every tile waits for the node-table workgroups, whose
// fix-up rewrites populations that the tiles read, from inputs the tiles
// overwrite.  The node-table workgroups come first in the grid, are
// dispatched first and fit on the GPU at once (n_head <= CUs), so no
// workgroup waits for one that is not running.  The table code here has no
// in-register re-collision, so the kernel keeps the plain collide's
// register count and occupancy.
constexpr uint32_t SPIN_LIMIT = 1u << 19;   // polls of a bounded wait (~0.1 s)

// thread 0 polls *cnt (relaxed, so a poll invalidates no cache) until it
// reaches target, then acquires; the workgroup waits at the barrier
__device__ __forceinline__ void wait_count(Ctrl* __restrict__ ctrl, uint32_t* cnt, uint32_t target)
{
    if (threadIdx.x == 0) {
        uint32_t it = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++it > SPIN_LIMIT) { atomicOr(&ctrl->health, H_SYNC); break; }
            __builtin_amdgcn_s_sleep(8);
        }
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
    }
    __syncthreads();
}

// every thread of the workgroup has written what it should: count the
// workgroup in *cnt, visibly for the other agents' acquire
__device__ __forceinline__ void count_done(uint32_t* cnt)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(cnt, 1u);
    }
}

// one (bead, table node) item of a sparse box: the node's fluid velocity from
// the current populations
template <typename R>
__device__ __forceinline__ void table_item(const BoxDev* __restrict__ boxes, const int32_t* __restrict__ list,
                                           const R* A, const ChainArgs& ca, R* __restrict__ near_u,
                                           int4* __restrict__ near_c, int one_box, const BoxDev& one, int li,
                                           int item)
{
    const int bi = one_box >= 0 ? one_box : list[li];
    const BoxDev bx = one_box >= 0 ? one : boxes[bi];
    const int N = bx.N, L = bx.L;
    if (item >= N * NEAR) return;
    const int b = item / NEAR, q = item - b * NEAR;
    const uint64_t g = bx.bead_off + (uint64_t)b;
    const double Ld = (double)L, iL = bx.inv_L;
    const int n0 = nearest_of(ca.x[3 * g], L, Ld, iL), n1 = nearest_of(ca.x[3 * g + 1], L, Ld, iL),
              n2 = nearest_of(ca.x[3 * g + 2], L, Ld, iL);
    if (q == 0) near_c[g] = make_int4(n0, n1, n2, 0);
    const uint32_t node = node_of(n0 - 1 + q % 3, n1 - 1 + (q / 3) % 3, n2 - 1 + q / 9, L);
    const uint32_t nz = node / ((uint32_t)L * (uint32_t)L), rem = node - nz * (uint32_t)L * (uint32_t)L;
    const uint32_t ny = rem / (uint32_t)L, nx = rem - ny * (uint32_t)L;
    R d[19];
    gather_pre<R, false>(A + bx.pop_off, Upwind(nx, ny, nz, (uint32_t)L), d);
    R u[3];
    node_velocity<R>(d, bx.rho0, 1.0 / bx.tau_lb, u);
    R* o = near_u + (g * NEAR + (uint64_t)q) * 3;
    o[0] = u[0]; o[1] = u[1]; o[2] = u[2];
}

template <typename R, int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, W))) void k_collide_headed(
    const BoxDev* __restrict__ boxes, const CollideConst<R>* __restrict__ ccs, const uint32_t* __restrict__ tile_box,
    R* A, R* B, Ctrl* __restrict__ ctrl, uint32_t s_off, const uint32_t* __restrict__ defer, uint32_t n_head,
    uint32_t head_x, const int32_t* __restrict__ list, ChainArgs ca, R* __restrict__ near_u,
    int4* __restrict__ near_c, const int32_t* __restrict__ bead_box, uint32_t* __restrict__ claim,
    const R* Aprev, int one_box, BoxDev one)   // Aprev and B are one buffer: the fix-up reads it, the tiles write it
{
    const uint32_t t = ctrl->step + s_off;
    const bool pend = ctrl->ovf_flag[(t - 1u) & 1u] == defer_stamp(t - 1u);
    if (blockIdx.x < n_head) {
        const uint32_t li = blockIdx.x / head_x, bx_ = blockIdx.x - li * head_x;
        if (pend) {
            // the workgroups of list entry li fix the listed nodes of its box:
            // the box and its constants stay uniform (scalar registers)
            const int bi = __builtin_amdgcn_readfirstlane(one_box >= 0 ? one_box : list[li]);
            const BoxDev& bx = boxes[bi];
            const uint32_t n_pend = min(ctrl->ovf_cnt, ca.ovf_cap);
            for (uint32_t e = bx_ * 256u + threadIdx.x; e < n_pend; e += head_x * 256u) {
                const uint64_t g = ca.ovf[2 * (uint64_t)e];
                const uint32_t r = ca.ovf[2 * (uint64_t)e + 1];
                if (bead_box[g] == bi)
                    fixup_node_claim_first<R>(bx, ccs, bi, r, ca.imp, claim, Aprev, A, ctrl, t - 1u);
            }
            count_done(&ctrl->head_fix[t & 1u]);
            wait_count(ctrl, &ctrl->head_fix[t & 1u], n_head);
        }
        table_item<R>(boxes, list, A, ca, near_u, near_c, one_box, one, (int)li, (int)(bx_ * 256u + threadIdx.x));
        count_done(&ctrl->head_done[t & 1u]);
        return;
    }
    if (pend) wait_count(ctrl, &ctrl->head_done[t & 1u], n_head);
    collide_tile<R>(boxes, ccs, tile_box, -1, blockIdx.x - n_head, A, B, ctrl, t, defer, threadIdx.x);
}

// one substep of one bead, as k_spread reads it
constexpr int REC = 8;   // doubles: fraction x3, coupling force x3, base node, unused

template <typename R>
__global__ __launch_bounds__(WG_MAXB) void k_chain_wg(const BoxDev* __restrict__ boxes,
                                                      const int32_t* __restrict__ list,
                                                      const R* __restrict__ A, ChainArgs ca,
                                                      const R* __restrict__ near_u,
                                                      const int4* __restrict__ near_c,
                                                      double* __restrict__ rec, Ctrl* __restrict__ ctrl,
                                                      uint32_t s_off, const int32_t* __restrict__ ca_bead_box,
                                                      int clear_ovf, uint32_t wait_head, int stamp_next)
{
    __shared__ double xs[3 * WG_MAXB];           // current positions
    __shared__ double x0s[3 * WG_MAXB];          // positions at the last list build
    __shared__ uint16_t nls[NL_SLOTS * WG_MAXB];  // neighbour k of bead b at [k * WG_MAXB + b]
    __shared__ uint32_t bk_cnt[NBK];             // list build: beads per cell bucket,
    __shared__ uint32_t bk_wsum[WG_MAXB / 64];   //   per-wave totals of the scan,
    __shared__ uint16_t bk_start[NBK + 1];       //   first slot of each bucket,
    __shared__ uint16_t bk_bead[WG_MAXB];        //   beads ordered by bucket,
    __shared__ float bk_pos[3 * WG_MAXB];        //   and their positions wrapped into the box
    __builtin_amdgcn_s_setprio(3);   // latency-bound chain beside the bandwidth-bound collide
    const int bi = list[blockIdx.x];
    const BoxDev& bx = boxes[bi];
    const int N = bx.N;
    const int b = (int)threadIdx.x;
    const bool act = b < N;
    const uint64_t g = bx.bead_off + (uint64_t)(act ? b : 0);
    const ChainSpan sp = chain_span(bx, act ? b : 0);
    const uint32_t t = ctrl->step + s_off;
    const int L = bx.L;
    const double Ld = (double)L, iL = bx.inv_L;
    const double dt = bx.dt, hdt_m = 0.5 * dt / bx.mass;
    const double eps24 = 24.0 * bx.eps;
    const double rl = sqrt(bx.rc2) + NL_SKIN;
    const double rl2 = rl * rl;
    const int nl_cap = ca.nl_cap < NL_SLOTS ? ca.nl_cap : NL_SLOTS;

    if (wait_head) {
        // the node tables come from the first workgroups of this step's
        // collide, which starts once the previous collide is done
        wait_count(ctrl, &ctrl->head_done[t & 1u], wait_head);
        if (b == 0) {   // the previous step's readers of its counts are done
            ctrl->head_done[(t + 1u) & 1u] = 0u;
            ctrl->head_fix[(t + 1u) & 1u] = 0u;
        }
    }
    if (clear_ovf) {
        // the previous step's impulses outside its deferred tiles were fixed
        // up by the node-table work, which left them in the field: clear
        // them before this step's spread, then reset both list counts
        const uint32_t n_ovf = min(ctrl->ovf_cnt, ca.ovf_cap);
        for (uint32_t e = (uint32_t)b; e < n_ovf; e += WG_MAXB) {
            const uint64_t gg = ca.ovf[2 * (uint64_t)e];
            const uint32_t r = ca.ovf[2 * (uint64_t)e + 1];
            unsigned long long* q = ca.imp + 3 * (boxes[ca_bead_box[gg]].node_off + r);
            q[0] = 0ull; q[1] = 0ull; q[2] = 0ull;
        }
        __syncthreads();   // every thread has read the count
        if (b == 0) { ctrl->ovf_cnt = 0u; ctrl->defer_cnt = 0u; }
    }

    double x[3] = {0, 0, 0}, v[3] = {0, 0, 0}, f[3] = {0, 0, 0};
    int nl_n = -2;
    int4 nc = make_int4(0, 0, 0, 0);
    if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[c] = ca.x[3 * g + c]; v[c] = ca.v[3 * g + c]; f[c] = ca.f[3 * g + c];
            x0s[3 * b + c] = ca.nl_x0[3 * g + c];
        }
        nc = near_c[g];
        nl_n = ca.nl_cnt[g];
        for (int k = 0; k < (nl_n > 0 ? nl_n : 0); ++k) nls[k * WG_MAXB + b] = ca.nl_idx[g * ca.nl_cap + k];
    }
    int rebuilds = 0;
    int cb0 = -1, cb1 = -1, cb2 = -1;   // base cell of the cached stencil
    R cu[8][3];                          // its node velocities (MD units), storage precision
    uint32_t hbits = 0;
    int tcnt = 0;

    for (int s = 0; s < bx.substeps; ++s) {
        if (act) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v[c] += f[c] * hdt_m;
                x[c] += v[c] * dt;
            }
        }
        __syncthreads();   // every read of xs by the previous substep is done
        bool rebuild = false;
        if (act) {
            xs[3 * b] = x[0]; xs[3 * b + 1] = x[1]; xs[3 * b + 2] = x[2];
            const double e0 = x[0] - x0s[3 * b], e1 = x[1] - x0s[3 * b + 1], e2 = x[2] - x0s[3 * b + 2];
            rebuild = nl_n == -2 || e0 * e0 + e1 * e1 + e2 * e2 > 0.25 * NL_SKIN * NL_SKIN;
        }
        // one bead past half the skin rebuilds every list; also publishes xs
        rebuild = __syncthreads_or(rebuild);
        if (rebuild) {
            ++rebuilds;
            int cnt = 0;
            // scan over every bead (boxes under three list radii across):
            // partner j joins the list when its minimum-image distance is
            // below the list radius
            auto consider = [&](int j) {
                double d0 = x[0] - xs[3 * j], d1 = x[1] - xs[3 * j + 1], d2 = x[2] - xs[3 * j + 2];
                d0 -= Ld * rint(d0 * iL); d1 -= Ld * rint(d1 * iL); d2 -= Ld * rint(d2 * iL);
                if (d0 * d0 + d1 * d1 + d2 * d2 < rl2) {
                    if (cnt < nl_cap) nls[cnt * WG_MAXB + b] = (uint16_t)j;
                    ++cnt;
                }
            };
            const int nc = list_cells(L, rl);
            if (nc >= 3) {
                // beads binned by cell bucket (counting sort in LDS), then each
                // bead visits the 27 buckets around its own cell
                int cc[3] = {0, 0, 0}, slot = 0, hb = 0;
                float pb[3] = {0.f, 0.f, 0.f};   // own position wrapped into [0, L)
                if (act) {
                    const double scl = (double)nc / Ld;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        double xt = x[c] - Ld * floor(x[c] * iL);
                        if (xt < 0.0) xt += Ld;
                        if (xt >= Ld) xt -= Ld;
                        const int q = (int)(xt * scl);
                        cc[c] = q < 0 ? 0 : (q >= nc ? nc - 1 : q);
                        pb[c] = (float)xt;
                    }
                    hb = bucket_of(cc[0], cc[1], cc[2]);
                }
                for (int i = b; i < NBK; i += WG_MAXB) bk_cnt[i] = 0u;
                __syncthreads();
                if (act) slot = (int)atomicAdd(&bk_cnt[hb], 1u);
                __syncthreads();
                // exclusive prefix sum of the bucket counts, four per thread: a
                // scan per wave, then the totals of the waves before
                static_assert(NBK == 4 * WG_MAXB, "four buckets per thread");
                uint32_t vb[4], vs = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) { vb[u] = bk_cnt[4 * b + u]; vs += vb[u]; }
                uint32_t inc = vs;
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t t = __shfl_up(inc, o, 64);
                    if ((b & 63) >= o) inc += t;
                }
                if ((b & 63) == 63) bk_wsum[b >> 6] = inc;
                __syncthreads();
                {
                    uint32_t base = 0;
                    for (int w = 0; w < (b >> 6); ++w) base += bk_wsum[w];
                    uint32_t ex = base + inc - vs;
#pragma unroll
                    for (int u = 0; u < 4; ++u) { bk_start[4 * b + u] = (uint16_t)ex; ex += vb[u]; }
                    if (b == WG_MAXB - 1) bk_start[NBK] = (uint16_t)ex;
                }
                __syncthreads();
                if (act) {
                    const int sl = bk_start[hb] + slot;
                    bk_bead[sl] = (uint16_t)b;
                    bk_pos[3 * sl] = pb[0]; bk_pos[3 * sl + 1] = pb[1]; bk_pos[3 * sl + 2] = pb[2];
                }
                __syncthreads();
                if (act) {
                    const float Lf = (float)Ld;
                    const float rlf2 = (float)((rl + NL_FP32_MARGIN) * (rl + NL_FP32_MARGIN));
                    for (int dz = -1; dz <= 1; ++dz) {
                        const int rz = cc[2] + dz, qz = wrap_cell(rz, nc);
                        // the neighbour cell's image next to this bead
                        const float oz = pb[2] + (rz < 0 ? Lf : (rz >= nc ? -Lf : 0.f));
                        for (int dy = -1; dy <= 1; ++dy) {
                            const int ry = cc[1] + dy, qy = wrap_cell(ry, nc);
                            const float oy = pb[1] + (ry < 0 ? Lf : (ry >= nc ? -Lf : 0.f));
#pragma unroll 1
                            for (int dx = -1; dx <= 1; ++dx) {
                                const int rx = cc[0] + dx;
                                const float ox = pb[0] + (rx < 0 ? Lf : (rx >= nc ? -Lf : 0.f));
                                const int q = bucket_of(wrap_cell(rx, nc), qy, qz);
                                const int k1 = bk_start[q + 1];
                                // four candidates per pass: their loads overlap
                                for (int k = bk_start[q]; k < k1; k += 4) {
                                    int jj[4];
                                    float r2[4];
#pragma unroll
                                    for (int u = 0; u < 4; ++u) {
                                        const bool ok = k + u < k1;
                                        const int sl = ok ? k + u : k;
                                        jj[u] = ok ? (int)bk_bead[sl] : b;
                                        const float d0 = bk_pos[3 * sl] - ox, d1 = bk_pos[3 * sl + 1] - oy,
                                                    d2 = bk_pos[3 * sl + 2] - oz;
                                        r2[u] = jj[u] == b ? rlf2 : d0 * d0 + d1 * d1 + d2 * d2;
                                    }
#pragma unroll
                                    for (int u = 0; u < 4; ++u)
                                        if (r2[u] < rlf2) {
                                            if (cnt < nl_cap) nls[cnt * WG_MAXB + b] = (uint16_t)jj[u];
                                            ++cnt;
                                        }
                                }
                            }
                        }
                    }
                    // ascending partner order, as a scan over all beads gives
                    if (cnt <= nl_cap)
                        for (int i = 1; i < cnt; ++i) {
                            const uint16_t key = nls[i * WG_MAXB + b];
                            int k = i - 1;
                            while (k >= 0 && nls[k * WG_MAXB + b] > key) {
                                nls[(k + 1) * WG_MAXB + b] = nls[k * WG_MAXB + b];
                                --k;
                            }
                            nls[(k + 1) * WG_MAXB + b] = key;
                        }
                }
            } else if (act) {   // boxes under three list radii across: every bead
                for (int j = 0; j < N; ++j)
                    if (j != b) consider(j);
            }
            if (act) {
                const int kept = cnt < nl_cap ? cnt : nl_cap;
                for (int k = 0; k < kept; ++k) ca.nl_idx[g * ca.nl_cap + k] = nls[k * WG_MAXB + b];
                nl_n = cnt > nl_cap ? -1 : cnt;   // -1: overflow, the full loop is used
                ca.nl_cnt[g] = nl_n;
#pragma unroll
                for (int c = 0; c < 3; ++c) { x0s[3 * b + c] = x[c]; ca.nl_x0[3 * g + c] = x[c]; }
            }
        }
        if (act) {
            // stencil first: the last force is dead after the drift
            double fr[3];
            const int i0 = cell_of(x[0], L, Ld, iL, fr[0]), i1 = cell_of(x[1], L, Ld, iL, fr[1]),
                      i2 = cell_of(x[2], L, Ld, iL, fr[2]);
            if (i0 != cb0 || i1 != cb1 || i2 != cb2) {
                cb0 = i0; cb1 = i1; cb2 = i2;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const uint32_t node = node_of(cb0 + (k & 1), cb1 + ((k >> 1) & 1), cb2 + ((k >> 2) & 1), L);
                    if (tcnt < ca.touch_cap) ca.touched[g * ca.touch_cap + tcnt] = node;
                    else hbits |= H_TABLE;
                    ++tcnt;
                }
                // offset of the base cell in the bead's 3x3x3 table: the
                // stencil lies inside it when the base cell is the nearest
                // node or the one below, on every axis
                int d0 = cb0 - nc.x + 1, d1 = cb1 - nc.y + 1, d2 = cb2 - nc.z + 1;
                d0 = d0 < 0 ? d0 + L : (d0 >= L ? d0 - L : d0);
                d1 = d1 < 0 ? d1 + L : (d1 >= L ? d1 - L : d1);
                d2 = d2 < 0 ? d2 + L : (d2 >= L ? d2 - L : d2);
                if (d0 <= 1 && d1 <= 1 && d2 <= 1) {
                    const R* tb = near_u + g * NEAR * 3;
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const int q = (d0 + (k & 1)) + 3 * (d1 + ((k >> 1) & 1)) + 9 * (d2 + ((k >> 2) & 1));
                        cu[k][0] = tb[3 * q]; cu[k][1] = tb[3 * q + 1]; cu[k][2] = tb[3 * q + 2];
                    }
                } else {   // moved past the table within this LB step: read the populations
                    const int i0v[3] = {cb0, cb1, cb2};
                    stencil_velocities<R, R, 1>(A + bx.pop_off, i0v, L, bx.rho0, 1.0 / bx.tau_lb, cu);
                }
            }
            double F[3] = {0, 0, 0};
            if (nl_n >= 0) {
                auto jof = [&](int k) { return (int)nls[k * WG_MAXB + b]; };
                for (int k = 0; k < nl_n; k += 4) wca_add4(x, xs, jof, k, nl_n, 1, b, Ld, iL, bx.rc2, bx.sigsq, eps24, F);
            } else {
                auto jof = [](int k) { return k; };
                for (int j = 0; j < N; j += 4) wca_add4(x, xs, jof, j, N, 1, b, Ld, iL, bx.rc2, bx.sigsq, eps24, F);
            }
            double Ff[3] = {0, 0, 0};
            hbits |= fene_force(bx, b, sp, x, xs, Ff);
            F[0] = Ff[0] + F[0]; F[1] = Ff[1] + F[1]; F[2] = Ff[2] + F[2];
            double ub[3] = {0, 0, 0};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const double wk = ((k & 1) ? fr[0] : 1.0 - fr[0]) * (((k >> 1) & 1) ? fr[1] : 1.0 - fr[1]) *
                                  (((k >> 2) & 1) ? fr[2] : 1.0 - fr[2]);
                ub[0] += wk * (double)cu[k][0]; ub[1] += wk * (double)cu[k][1]; ub[2] += wk * (double)cu[k][2];
            }
            const U4 w = philox10(U4{(uint32_t)b, t, (1u << 16) | (uint32_t)s, 0u}, bx.seed, bx.box_id);
            const uint32_t ws[3] = {w.x, w.y, w.z};
            double fcl[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double ffr = -bx.zeta * (v[c] - ub[c]);
                const double frn = bx.bead_noise * unit_noise<double>(ws[c]);
                fcl[c] = ffr + frn;
                f[c] = F[c] + fcl[c];
                v[c] += f[c] * hdt_m;
            }
            double* r = rec + ((uint64_t)s * ca.total_beads + g) * REC;
            r[0] = fr[0]; r[1] = fr[1]; r[2] = fr[2];
            r[3] = fcl[0]; r[4] = fcl[1]; r[5] = fcl[2];
            r[6] = (double)node_of(cb0, cb1, cb2, L);
            if (s + 1 == bx.substeps) {
#pragma unroll
                for (int c = 0; c < 3; ++c) ca.fc[3 * g + c] = fcl[c];
            }
        }
    }
    if (act) {
        ca.touched_cnt[g] = tcnt < ca.touch_cap ? tcnt : ca.touch_cap;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ca.x[3 * g + c] = x[c]; ca.v[3 * g + c] = v[c]; ca.f[3 * g + c] = f[c];
        }
        if (stamp_next && ca.defer) {
            // the next step's deferred tiles: those of the table around the
            // nearest node of the end position (what its node-table work uses)
            const int m0 = nearest_of(x[0], L, Ld, iL), m1 = nearest_of(x[1], L, Ld, iL),
                      m2 = nearest_of(x[2], L, Ld, iL);
            const uint32_t sn = defer_stamp(t + 1u);
            for (int q = 0; q < NEAR; ++q) {
                const uint32_t node = node_of(m0 - 1 + q % 3, m1 - 1 + (q / 3) % 3, m2 - 1 + q / 9, L);
                ca.defer[2u * dseg_of(bx, node) + (sn & 1u)] = sn;
            }
        }
        if (ca.vhist) {
            double* hv = ca.vhist + ((uint64_t)(t % (uint32_t)ca.hist_len) * ca.total_beads + g) * 3;
            hv[0] = v[0]; hv[1] = v[1]; hv[2] = v[2];
        }
        if (hbits) atomicOr(&ctrl->health, hbits);
    }
    if (b == 0 && rebuilds) atomicAdd(&ca.nl_rebuilds[bi], (uint32_t)rebuilds);
}

// an impulse on a node whose tile is not deferred (the bead left its table):
// listed for the end-of-step fix-up
__device__ __forceinline__ uint32_t list_overflow(const ChainArgs& ca, const BoxDev& bx, uint64_t g, uint32_t node,
                                                  Ctrl* __restrict__ ctrl, uint32_t stamp)
{
    if (!ca.defer || ca.defer[2u * dseg_of(bx, node) + (stamp & 1u)] == stamp) return 0u;
    ca.ovm[bx.node_off + node] = stamp;   // read by the next step's node-table work
    ctrl->ovf_flag[stamp & 1u] = stamp;   // the next step's collide waits for that work
    const uint32_t k = atomicAdd(&ctrl->ovf_cnt, 1u);
    if (k >= ca.ovf_cap) return H_TABLE;
    ca.ovf[2 * (uint64_t)k] = (uint32_t)g;
    ca.ovf[2 * (uint64_t)k + 1] = node;
    return 0u;
}

// node impulses from the substep records: thread (bead, corner k) accumulates
// -w_k (F_fric + F_rand) dt over the substeps that share a stencil, in MD
// units and in substep order, and hands each stencil's sum over when the
// stencil changes and after the last substep (lattice units, fixed point)
__global__ __launch_bounds__(256) void k_spread(const BoxDev* __restrict__ boxes, const int32_t* __restrict__ list,
                                                ChainArgs ca, const double* __restrict__ rec,
                                                Ctrl* __restrict__ ctrl, uint32_t s_off)
{
    const BoxDev& bx = boxes[list[blockIdx.y]];
    if (bx.dense) return;   // binned and gathered instead (k_bin_runs, k_gather_imp)
    const int N = bx.N, L = bx.L;
    const int tid = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (tid >= N * 8) return;
    const int b = tid >> 3, k = tid & 7;
    const uint64_t g = bx.bead_off + (uint64_t)b;
    const double dt = bx.dt, tau = bx.tau_lb;
    const uint32_t stamp = defer_stamp(ctrl->step + s_off);
    unsigned long long* imp = ca.imp + 3 * bx.node_off;
    uint32_t hb = 0;
    double acc[3] = {0, 0, 0};
    uint32_t cur = 0xffffffffu;
    for (int s = 0; s < bx.substeps; ++s) {
        const double* r = rec + ((uint64_t)s * ca.total_beads + g) * REC;
        const uint32_t base = (uint32_t)r[6];
        const uint32_t bz = base / ((uint32_t)L * (uint32_t)L), rem = base - bz * (uint32_t)L * (uint32_t)L;
        const uint32_t by = rem / (uint32_t)L, bxn = rem - by * (uint32_t)L;
        const uint32_t node = node_of((int)bxn + (k & 1), (int)by + ((k >> 1) & 1), (int)bz + ((k >> 2) & 1), L);
        if (node != cur) {
            if (cur != 0xffffffffu) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double q = acc[c] * tau;
                    if (!(fabs(q) < IMP_MAX)) { hb |= H_FIXED; q = 0.0; }
                    atomicAdd(imp + 3 * (uint64_t)cur + c, (unsigned long long)(long long)llrint(q * IMP_SCALE));
                }
                hb |= list_overflow(ca, bx, g, cur, ctrl, stamp);
            }
            cur = node;
            acc[0] = acc[1] = acc[2] = 0.0;
        }
        const double wk = ((k & 1) ? r[0] : 1.0 - r[0]) * (((k >> 1) & 1) ? r[1] : 1.0 - r[1]) *
                          (((k >> 2) & 1) ? r[2] : 1.0 - r[2]);
        acc[0] -= wk * r[3] * dt;
        acc[1] -= wk * r[4] * dt;
        acc[2] -= wk * r[5] * dt;
    }
    if (cur != 0xffffffffu) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double q = acc[c] * tau;
            if (!(fabs(q) < IMP_MAX)) { hb |= H_FIXED; q = 0.0; }
            atomicAdd(imp + 3 * (uint64_t)cur + c, (unsigned long long)(long long)llrint(q * IMP_SCALE));
        }
        hb |= list_overflow(ca, bx, g, cur, ctrl, stamp);
    }
    if (hb) atomicOr(&ctrl->health, hb);
}

// Dense boxes hand their impulses over without atomics.  A stencil run is a
// maximal range of substeps in which a bead keeps one base node; k_spread
// accumulates each (run, corner) in FP64 and rounds it to fixed point once.
// Here k_bin_runs gives every run a slot, the slots sorted by base node
// (counting sort in LDS, one workgroup per box); k_run_impulse, one thread
// per (bead, corner) like k_spread, stores each (run, corner) value in its
// run's slot; k_gather_imp gives each node the sum over the runs whose
// stencil holds it.  The fixed-point sums do not depend on order, so the
// field equals the one the atomics would build.
constexpr uint32_t DENSE_MAXV = 32768;   // a dense box has at most 32 N <= 32768 nodes
__global__ __launch_bounds__(WG_MAXB) void k_bin_runs(const BoxDev* __restrict__ boxes,
                                                      const int32_t* __restrict__ list, ChainArgs ca,
                                                      const double* __restrict__ rec,
                                                      uint32_t* __restrict__ bin_start,
                                                      uint32_t* __restrict__ slot_of)
{
    __shared__ uint32_t cnt[DENSE_MAXV];        // runs per base node, then the placement cursor
    __shared__ uint32_t wsum[WG_MAXB / 64];
    const BoxDev& bx = boxes[list[blockIdx.x]];
    if (!bx.dense) return;
    const int N = bx.N, S = bx.substeps, L = bx.L;
    const uint32_t V = (uint32_t)L * L * L;
    const int b = (int)threadIdx.x;
    const bool act = b < N;
    const uint64_t g = bx.bead_off + (uint64_t)(act ? b : 0);
    auto base_at = [&](int s) {
        return (uint32_t)rec[((uint64_t)s * ca.total_beads + g) * REC + 6];
    };
    for (uint32_t i = (uint32_t)b; i < V; i += WG_MAXB) cnt[i] = 0u;
    __syncthreads();
    if (act) {
        uint32_t cur = 0xffffffffu;
        for (int s = 0; s < S; ++s) {
            const uint32_t base = base_at(s);
            if (base != cur) { atomicAdd(&cnt[base], 1u); cur = base; }
        }
    }
    __syncthreads();
    // exclusive prefix sum over the V counts: a chunk of C per thread, a
    // scan per wave of the chunk totals, then the totals of the waves before
    const uint32_t C = (V + WG_MAXB - 1) / WG_MAXB;
    const uint32_t i0 = (uint32_t)b * C < V ? (uint32_t)b * C : V, i1 = i0 + C < V ? i0 + C : V;
    uint32_t tot = 0;
    for (uint32_t i = i0; i < i1; ++i) tot += cnt[i];
    uint32_t inc = tot;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o, 64);
        if ((b & 63) >= o) inc += t;
    }
    if ((b & 63) == 63) wsum[b >> 6] = inc;
    __syncthreads();
    uint32_t run = inc - tot;
    for (int w = 0; w < (b >> 6); ++w) run += wsum[w];
    uint32_t* bs = bin_start + bx.bin_off;
    for (uint32_t i = i0; i < i1; ++i) {
        const uint32_t c = cnt[i];
        bs[i] = run;
        cnt[i] = run;
        run += c;
    }
    if (b == WG_MAXB - 1) bs[V] = run;
    __syncthreads();
    if (act) {
        // slot of the j-th run of bead b
        uint32_t cur = 0xffffffffu;
        int j = 0;
        for (int s = 0; s < S; ++s) {
            const uint32_t base = base_at(s);
            if (base != cur) {
                slot_of[bx.item_off + (uint64_t)b * S + j] = atomicAdd(&cnt[base], 1u);
                ++j;
                cur = base;
            }
        }
    }
}

// one thread per (bead, corner): k_spread's accumulation, stored in the
// run's slot instead of added to the field
__global__ __launch_bounds__(256) void k_run_impulse(const BoxDev* __restrict__ boxes,
                                                     const int32_t* __restrict__ list, ChainArgs ca,
                                                     const double* __restrict__ rec,
                                                     const uint32_t* __restrict__ slot_of,
                                                     unsigned long long* __restrict__ runimp,
                                                     Ctrl* __restrict__ ctrl)
{
    const BoxDev& bx = boxes[list[blockIdx.y]];
    if (!bx.dense) return;
    const int N = bx.N, S = bx.substeps;
    const int tid = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (tid >= N * 8) return;
    const int b = tid >> 3, k = tid & 7;
    const uint64_t g = bx.bead_off + (uint64_t)b;
    const double dt = bx.dt, tau = bx.tau_lb;
    uint32_t hb = 0;
    double acc[3] = {0, 0, 0};
    uint32_t cur = 0xffffffffu;
    int j = 0;
    auto store = [&]() {
        unsigned long long* o = runimp + (bx.item_off + slot_of[bx.item_off + (uint64_t)b * S + j]) * 24 + 3 * k;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double q = acc[c] * tau;
            if (!(fabs(q) < IMP_MAX)) { hb |= H_FIXED; q = 0.0; }
            o[c] = (unsigned long long)(long long)llrint(q * IMP_SCALE);
        }
    };
    for (int s = 0; s < S; ++s) {
        const double* r = rec + ((uint64_t)s * ca.total_beads + g) * REC;
        const uint32_t base = (uint32_t)r[6];
        if (base != cur) {
            if (cur != 0xffffffffu) { store(); ++j; }
            cur = base;
            acc[0] = acc[1] = acc[2] = 0.0;
        }
        const double wk = ((k & 1) ? r[0] : 1.0 - r[0]) * (((k >> 1) & 1) ? r[1] : 1.0 - r[1]) *
                          (((k >> 2) & 1) ? r[2] : 1.0 - r[2]);
        acc[0] -= wk * r[3] * dt;
        acc[1] -= wk * r[4] * dt;
        acc[2] -= wk * r[5] * dt;
    }
    if (cur != 0xffffffffu) store();
    if (hb) atomicOr(&ctrl->health, hb);
}

__global__ __launch_bounds__(256) void k_gather_imp(const BoxDev* __restrict__ boxes,
                                                    const int32_t* __restrict__ list, ChainArgs ca,
                                                    const uint32_t* __restrict__ bin_start,
                                                    const unsigned long long* __restrict__ runimp)
{
    const BoxDev& bx = boxes[list[blockIdx.y]];
    if (!bx.dense) return;
    const int L = bx.L;
    const uint32_t V = (uint32_t)L * L * L;
    const uint32_t r = blockIdx.x * 256u + threadIdx.x;
    if (r >= V) return;
    const int x = (int)(r % (uint32_t)L), y = (int)((r / (uint32_t)L) % (uint32_t)L), z = (int)(r / ((uint32_t)L * L));
    const uint32_t* bs = bin_start + bx.bin_off;
    // the bins of the 8 base nodes whose corner k is this node: all bounds
    // are loaded before any is used
    uint32_t e0[8], e1[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t base = node_of(x - (k & 1), y - ((k >> 1) & 1), z - ((k >> 2) & 1), L);
        e0[k] = bs[base];
        e1[k] = bs[base + 1];
    }
    unsigned long long sum[3] = {0ull, 0ull, 0ull};
#pragma unroll
    for (int k = 0; k < 8; ++k)
        for (uint32_t e = e0[k]; e < e1[k]; ++e) {
            const unsigned long long* q = runimp + (bx.item_off + e) * 24 + 3 * k;
            sum[0] += q[0]; sum[1] += q[1]; sum[2] += q[2];
        }
    unsigned long long* dst = ca.imp + 3 * (bx.node_off + r);
    dst[0] = sum[0]; dst[1] = sum[1]; dst[2] = sum[2];
}

// ---------------------------------------------------------------- fixup
// Collide node r of box bi with its impulse from the dense field and
// overwrite its streamed outputs.  The claim stamp makes one caller per node
// and step do it: the populations and the impulse are loaded before the
// claim returns, so the three latencies overlap.
template <typename R>
__device__ __forceinline__ void fixup_node(const FixBox& bx, const CollideConst<R>& cc, uint32_t r,
                                           unsigned long long* __restrict__ imp, uint32_t* __restrict__ claim,
                                           const R* __restrict__ A, R* __restrict__ B, Ctrl* __restrict__ ctrl,
                                           uint32_t t, int keep_imp)
{
    const uint64_t node = bx.node_off + r;
    const Upwind up = upwind_of(r, bx.L, bx.inv_L);
    R d[19];
    gather_pre<R, false>(A + bx.pop_off, up, d);
    unsigned long long* q = imp + 3 * node;
    const unsigned long long q0 = q[0], q1 = q[1], q2 = q[2];
    if (atomicExch(&claim[node], t + 1u) == t + 1u) return;   // another caller took this node
    if (!keep_imp) { q[0] = 0ull; q[1] = 0ull; q[2] = 0ull; }
    const R fx = (R)((double)(long long)q0 * IMP_INV_SCALE), fy = (R)((double)(long long)q1 * IMP_INV_SCALE),
            fz = (R)((double)(long long)q2 * IMP_INV_SCALE);
    R o[19];
    const uint32_t h = collide<R>(d, o, fx, fy, fz, cc, r, t, bx.seed, bx.box_id);
    R* b = B + bx.pop_off;
#pragma unroll
    for (int i = 0; i < 19; ++i) b[pop_at(i, r)] = o[i];
    if (h) atomicOr(&ctrl->health, h);
}

// FIX_LANES threads per launched bead; thread j fixes the bead's touched-node
// slots j, j + FIX_LANES, ... (a bead that keeps its cell fills 8 slots, so
// one pass is the rule).  A node touched by several beads is fixed once
// (claim stamp).  skip_big: the beads of chains above BIG_CHAIN have their
// nodes in deferred tiles or in the overflow list.
constexpr int FIX_LANES = 16;   // <= touch_cap = 8 (substeps + 1)
template <typename R>
__global__ __launch_bounds__(256) void k_fixup(const BoxDev* __restrict__ boxes,
                                               const CollideConst<R>* __restrict__ ccs,
                                               const int32_t* __restrict__ bead_box, uint64_t bead0,
                                               uint32_t n_entries, ChainArgs ca, uint32_t* __restrict__ claim,
                                               const R* __restrict__ A, R* __restrict__ B,
                                               Ctrl* __restrict__ ctrl, uint32_t s_off, int keep_imp, int skip_big)
{
    const uint32_t e = blockIdx.x * 256u + threadIdx.x;
    if (e >= n_entries) return;
    const uint64_t g = bead0 + e / (uint32_t)FIX_LANES;
    const int j = (int)(e % (uint32_t)FIX_LANES);
    // independent loads together: the slot count, the box, the first slot
    // (read for every thread, used below the count) and the step; then, in
    // one more round, every field of the box and its collision constants
    const int cnt = ca.touched_cnt[g];
    const int bi = bead_box[g];
    const uint32_t r0 = ca.touched[g * ca.touch_cap + j];
    const uint32_t t = ctrl->step + s_off;
    const BoxDev& bx = boxes[bi];
    const FixBox fb = fix_box(bx);
    const int dense = bx.dense, nb = bx.N;
    const CollideConst<R> cc = ccs[bi];
    // a dense box's collide takes the impulses itself
    // (one test, so that no load waits for another's branch; the empty asm
    // keeps the box fields' loads above it, beside the tested ones)
    asm volatile("" ::"v"(fb.L), "v"(fb.pop_off), "v"(fb.node_off), "v"(fb.inv_L), "v"(fb.seed), "v"(fb.box_id));
    if ((j >= cnt) | (dense != 0) | ((skip_big != 0) & (nb > BIG_CHAIN))) return;
    fixup_node<R>(fb, cc, r0, ca.imp, claim, A, B, ctrl, t, keep_imp);
    for (int k = j + FIX_LANES; k < cnt; k += FIX_LANES)
        fixup_node<R>(fb, cc, ca.touched[g * ca.touch_cap + k], ca.imp, claim, A, B, ctrl, t, keep_imp);
}

// End of a step that deferred tiles (one workgroup): fix the listed nodes
// outside the deferred tiles, then reset both list counts for the next step
// (the per-tile stamps need no clearing).  Runs after the plain collide, the
// deferred tiles' collide and the coupling.
template <typename R>
__global__ __launch_bounds__(256) void k_overflow(const BoxDev* __restrict__ boxes,
                                                   const CollideConst<R>* __restrict__ ccs,
                                                   const int32_t* __restrict__ bead_box, ChainArgs ca,
                                                   uint32_t* __restrict__ claim, const R* __restrict__ A,
                                                   R* __restrict__ B, Ctrl* __restrict__ ctrl, uint32_t s_off,
                                                   uint32_t advance)
{
    const uint32_t t = ctrl->step + s_off;
    const uint32_t n_ovf = min(ctrl->ovf_cnt, ca.ovf_cap);
    for (uint32_t e = threadIdx.x; e < n_ovf; e += blockDim.x) {
        const uint64_t g = ca.ovf[2 * (uint64_t)e];
        const uint32_t r = ca.ovf[2 * (uint64_t)e + 1];
        const int bi = bead_box[g];
        fixup_node<R>(fix_box(boxes[bi]), ccs[bi], r, ca.imp, claim, A, B, ctrl, t, 0);
    }
    __syncthreads();   // every thread has read the count and the step
    if (threadIdx.x == 0) {
        ctrl->defer_cnt = 0u;
        ctrl->ovf_cnt = 0u;
        ctrl->step += advance;   // the run's steps, when this kernel ends it (else 0)
    }
}

// Collide and stream one 256-node tile after the coupling stage: each node's
// impulse comes straight from the fixed-point field, which is cleared where
// it was set.  Same arithmetic as the fix-up, over a whole tile.
template <typename R>
__device__ __forceinline__ void collide_forced_tile(const BoxDev* __restrict__ boxes,
                                                    const CollideConst<R>* __restrict__ ccs,
                                                    const uint32_t* __restrict__ tile_box, int fixed_box,
                                                    uint32_t tile, unsigned long long* __restrict__ imp,
                                                    const R* __restrict__ A, R* __restrict__ B,
                                                    Ctrl* __restrict__ ctrl, uint32_t t, uint32_t lane)
{
    const int bi = fixed_box >= 0 ? fixed_box : (int)tile_box[tile];
    const BoxDev& bx = boxes[bi];
    const int L = bx.L;
    const uint32_t V = (uint32_t)L * L * L;
    const uint32_t r = (tile - bx.tile_begin) * 256u + lane;
    if (r >= V) return;
    const CollideConst<R> cc = ccs[bi];
    const Upwind up = upwind_of(r, L, bx.inv_L);
    R d[19];
    gather_pre<R, false>(A + bx.pop_off, up, d);
    unsigned long long* q = imp + 3 * (bx.node_off + r);
    const unsigned long long q0 = q[0], q1 = q[1], q2 = q[2];
    if (q0 | q1 | q2) { q[0] = 0ull; q[1] = 0ull; q[2] = 0ull; }
    const R fx = (R)((double)(long long)q0 * IMP_INV_SCALE), fy = (R)((double)(long long)q1 * IMP_INV_SCALE),
            fz = (R)((double)(long long)q2 * IMP_INV_SCALE);
    R o[19];
    const uint32_t h = collide<R>(d, o, fx, fy, fz, cc, r, t, bx.seed, bx.box_id);
    R* b = B + bx.pop_off;
#pragma unroll
    for (int i = 0; i < 19; ++i) __builtin_nontemporal_store(o[i], b + pop_at(i, r));
    if (h) atomicOr(&ctrl->health, h);
}

// every node of a dense box, after its coupling stage
template <typename R>
__global__ __launch_bounds__(256) void k_collide_forced(const BoxDev* __restrict__ boxes,
                                                        const CollideConst<R>* __restrict__ ccs,
                                                        const uint32_t* __restrict__ tile_box, int fixed_box,
                                                        uint32_t tile0, unsigned long long* __restrict__ imp,
                                                        const R* __restrict__ A, R* __restrict__ B,
                                                        Ctrl* __restrict__ ctrl, uint32_t s_off)
{
    collide_forced_tile<R>(boxes, ccs, tile_box, fixed_box, tile0 + blockIdx.x, imp, A, B, ctrl,
                           ctrl->step + s_off, threadIdx.x);
}

// The deferred tiles of a step as a list, built after the coupling on the
// chain's stream: thread (bead, table node) of a sparse box claims the node's
// tile for this step; each wave appends its new tiles with one atomic.
__global__ __launch_bounds__(256) void k_defer_list(const BoxDev* __restrict__ boxes,
                                                    const int32_t* __restrict__ list, ChainArgs ca,
                                                    const int4* __restrict__ near_c, Ctrl* __restrict__ ctrl,
                                                    uint32_t s_off)
{
    const BoxDev& bx = boxes[list[blockIdx.y]];
    if (bx.dense) return;
    const int tid = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const uint32_t stamp = defer_stamp(ctrl->step + s_off);
    bool win = false;
    uint32_t seg = 0;
    if (tid < bx.N * NEAR) {
        const int b = tid / NEAR, q = tid - b * NEAR;
        const int4 nc = near_c[bx.bead_off + (uint64_t)b];
        const uint32_t node = node_of(nc.x - 1 + q % 3, nc.y - 1 + (q / 3) % 3, nc.z - 1 + q / 9, bx.L);
        seg = dseg_of(bx, node);
        win = ca.dclaim[seg] != stamp && atomicExch(&ca.dclaim[seg], stamp) != stamp;
    }
    const unsigned long long m = __ballot(win);
    if (m == 0ull) return;
    const int lane = (int)(threadIdx.x & 63u);
    const int lead = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane == lead) base = atomicAdd(&ctrl->defer_cnt, (uint32_t)__popcll(m));
    base = __shfl(base, lead);
    if (win) {
        const uint32_t k = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (k < ca.defer_cap) ca.defer_list[k] = seg;
        else atomicOr(&ctrl->health, H_TABLE);
    }
}

// the deferred tiles of a step, after its coupling stage, beside the plain
// collide of the other tiles (both only read the current state and write
// disjoint nodes)
template <typename R>
__global__ __launch_bounds__(256) void k_collide_deferred(const BoxDev* __restrict__ boxes,
                                                          const CollideConst<R>* __restrict__ ccs,
                                                          const uint32_t* __restrict__ tile_box,
                                                          const uint32_t* __restrict__ defer_list, uint32_t cap,
                                                          unsigned long long* __restrict__ imp,
                                                          const R* __restrict__ A, R* __restrict__ B,
                                                          Ctrl* __restrict__ ctrl, uint32_t s_off)
{
    // one wavefront per listed segment
    const uint32_t t = ctrl->step + s_off;
    const uint32_t n = min(ctrl->defer_cnt, cap);
    // the wavefront index made uniform: the segment, its tile and box, and the
    // box constants then sit in scalar registers
    const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x / DSEG), lane = threadIdx.x % DSEG;
    for (uint32_t k = blockIdx.x * DSEG_PER_TILE + w; k < n; k += gridDim.x * DSEG_PER_TILE) {
        const uint32_t seg = defer_list[k];
        collide_forced_tile<R>(boxes, ccs, tile_box, -1, seg / DSEG_PER_TILE, imp, A, B, ctrl, t,
                               (seg % DSEG_PER_TILE) * DSEG + lane);
    }
}

// --------------------------------------------------------------- advance
__global__ void k_advance(Ctrl* ctrl, uint32_t n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ctrl->step += n;
}

// ----------------------------------------------------------------- stats
// Per tile of 256 nodes: FP64 sums of mass deviation, momentum, squared modes,
// negative population count.  Layout of a record: [0] sum drho, [1..3] j,
// [4] neg count, [5..23] sum m_k^2 (m of the deviations; m_0 = drho).
// Every sum is a fixed tree (butterfly within each wavefront, then the four
// wavefronts in order, then fixed chunks of a box's tiles, then the chunks in
// order), so a state gives the same bits on every call and in any batch.
constexpr int NSTAT = NSTAT_REC;

// value of v in another lane of the same 16-lane row, by a DPP lane move of
// both 32-bit halves (CTRL: a gfx9 DPP control; every source lane is active)
template <int CTRL>
__device__ __forceinline__ double dpp_from(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value(double v, int lane)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum of v[k] over the 64 lanes of a wavefront for k < NV, with every lane of
// the wavefront active: within each 16-lane row by DPP moves (neighbour in the
// pair, the other pair of the quad, the mirrored quad, the mirrored half-row;
// each stage adds the same two values in either order, so all 16 lanes hold
// the same row sum), then the four row sums in row order.  The NV sums are
// advanced stage by stage so that their moves issue back to back.  Every lane
// returns the same bits.
template <int NV>
__device__ __forceinline__ void wave_sums(double v[NV])
{
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += dpp_from<0xB1>(v[k]);    // quad_perm [1,0,3,2]
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += dpp_from<0x4E>(v[k]);    // quad_perm [2,3,0,1]
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += dpp_from<0x141>(v[k]);   // row_half_mirror
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += dpp_from<0x140>(v[k]);   // row_mirror
#pragma unroll
    for (int k = 0; k < NV; ++k)
        v[k] = ((lane_value(v[k], 0) + lane_value(v[k], 16)) + lane_value(v[k], 32)) + lane_value(v[k], 48);
}

// sum of acc[0..NV-1] over a 256-thread block (all threads active): per
// wavefront, then wavefronts 0..3 in order; the result is valid in threads
// 0..NV-1 (thread k holds sum k).  acc is consumed.
template <int NV>
__device__ __forceinline__ double block_sum256(double acc[NV], double (*lds)[NV])
{
    const int wv_ = threadIdx.x >> 6, ln = threadIdx.x & 63;
    wave_sums<NV>(acc);
    if (ln == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[wv_][k] = acc[k];
    }
    __syncthreads();
    double r = 0.0;
    if ((int)threadIdx.x < NV) r = ((lds[0][threadIdx.x] + lds[1][threadIdx.x]) + lds[2][threadIdx.x]) + lds[3][threadIdx.x];
    return r;
}

// grid (records of the largest box, boxes): block (c, box) sums tiles
// c*STAT_TPB .. c*STAT_TPB + STAT_TPB - 1 of the box, one node per thread and
// tile, into record stat_off + c
__device__ __forceinline__ float uniform_value(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform_value(double v)
{
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                            __builtin_amdgcn_readfirstlane(__double2loint(v)));
}

// the pre-collision populations of node `up` with 32-bit offsets from the
// box's array (valid while that array is under 4 GiB): a uniform base and one
// 32-bit offset per load instead of 64-bit address arithmetic
template <typename R>
__device__ __forceinline__ void gather_pre32(const R* __restrict__ a, const Upwind& up, R d[19])
{
    const char* base = (const char*)a;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const uint32_t s = up.src(i);
        const uint32_t e = ((s >> PTILE_LOG) * 19u + (uint32_t)i) * PTILE + (s & (PTILE - 1u));
        d[i] = *(const R*)(base + (uint64_t)(e * (uint32_t)sizeof(R)));
    }
}

template <typename R, bool O32>
__global__ __launch_bounds__(256) void k_stats(const BoxDev* __restrict__ boxes, const R* __restrict__ A,
                                               double* __restrict__ part)
{
    __shared__ double red[4][NSTAT];
    const BoxDev& bx = boxes[blockIdx.y];
    const uint32_t c = blockIdx.x;
    if (c >= stat_recs_of(bx.n_tiles)) return;
    const uint32_t V = (uint32_t)bx.L * bx.L * bx.L;
    const R* a = A + bx.pop_off;
    // n_i = fl(w_i rho0) + delta_i (FP64) is negative exactly when delta_i
    // lies below -fl(w_i rho0): the rounded sum of two doubles keeps the sign
    // of the exact one.  For FP32 storage the test compares delta_i with the
    // smallest float not below that double, which decides the same; the
    // count is an integer.
    R thr[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const double cth = -(wv(i) * bx.rho0);
        R f = (R)cth;
        if ((double)f < cth) f = nextafter(f, (R)INFINITY);
        thr[i] = uniform_value(f);   // the same in every lane: kept in scalar registers
    }
    double acc[NSTAT];
#pragma unroll
    for (int k = 0; k < NSTAT; ++k) acc[k] = 0.0;
    uint32_t neg = 0;
    for (int k = 0; k < STAT_TPB; ++k) {
        const uint32_t r = (c * STAT_TPB + k) * 256u + threadIdx.x;
        if (r >= V) break;
        const Upwind up = upwind_of(r, bx.L, bx.inv_L);
        R dr[19];
        if (O32) gather_pre32<R>(a, up, dr);
        else gather_pre<R, false>(a, up, dr);
        double d[19], m[19];
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            d[i] = (double)dr[i];
            neg += dr[i] < thr[i] ? 1u : 0u;
        }
        to_modes<double>(d, m);
        acc[0] += m[0]; acc[1] += m[1]; acc[2] += m[2]; acc[3] += m[3];
#pragma unroll
        for (int q = 0; q < 19; ++q) acc[5 + q] += m[q] * m[q];
    }
    acc[4] = (double)neg;   // what adding 1.0 per negative population gives, exactly
    const double s = block_sum256<NSTAT>(acc, red);
    if (threadIdx.x < NSTAT) part[(uint64_t)(bx.stat_off + c) * NSTAT + threadIdx.x] = s;
}

// grid (STAT_CHUNKS, boxes): block (c, box) sums the block records of chunk
// c of the box (a fixed split of its records into STAT_CHUNKS ranges)
__global__ __launch_bounds__(256) void k_stats_mid(const BoxDev* __restrict__ boxes,
                                                   const double* __restrict__ part, double* __restrict__ mid)
{
    __shared__ double red[4][NSTAT];
    const BoxDev& bx = boxes[blockIdx.y];
    const uint32_t nrec = stat_recs_of(bx.n_tiles);
    const uint32_t per = (nrec + STAT_CHUNKS - 1) / STAT_CHUNKS;
    const uint32_t t0 = blockIdx.x * per, t1 = min(nrec, t0 + per);
    double acc[NSTAT];
#pragma unroll
    for (int k = 0; k < NSTAT; ++k) acc[k] = 0.0;
    for (uint32_t tt = t0 + threadIdx.x; tt < t1; tt += 256) {
        const double* rec = part + (uint64_t)(bx.stat_off + tt) * NSTAT;
#pragma unroll
        for (int k = 0; k < NSTAT; ++k) acc[k] += rec[k];
    }
    const double s = block_sum256<NSTAT>(acc, red);
    if (threadIdx.x < NSTAT) mid[((uint64_t)blockIdx.y * STAT_CHUNKS + blockIdx.x) * NSTAT + threadIdx.x] = s;
}

// one wavefront per box: the box's STAT_CHUNKS chunk sums, in chunk order
__global__ __launch_bounds__(64) void k_stats_final(const double* __restrict__ mid, double* __restrict__ out)
{
    const int k = threadIdx.x;
    if (k >= NSTAT) return;
    const double* m = mid + (uint64_t)blockIdx.x * STAT_CHUNKS * NSTAT;
    double s = 0.0;
    for (int c = 0; c < STAT_CHUNKS; ++c) s += m[c * NSTAT + k];
    out[(uint64_t)blockIdx.x * NSTAT + k] = s;
}

// one block per box: chain sums.  Record: [0..2] sum x, [3..5] sum m v,
// [6..8] sum fc, [9] sum over the chains of R_e^2, then after the second pass
// [10] sum over beads of |x - com of the bead's chain|^2.
constexpr int NCHAIN = 11;

__global__ __launch_bounds__(256) void k_chain_obs(const BoxDev* __restrict__ boxes, ChainArgs ca,
                                                   double* __restrict__ out)
{
    __shared__ double red[4][9];
    __shared__ double red1[4][1];
    __shared__ double sums[9];
    __shared__ double ccom[3 * MAXB];   // per-chain centres of mass (several chains)
    const BoxDev& bx = boxes[blockIdx.x];
    const int N = bx.N;
    const int n = bx.chain_len, M = N > 0 ? N / n : 0;
    double acc[9];
    for (int k = 0; k < 9; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < N; b += 256) {
        const uint64_t g = bx.bead_off + b;
        for (int c = 0; c < 3; ++c) {
            acc[c] += ca.x[3 * g + c];
            acc[3 + c] += bx.mass * ca.v[3 * g + c];
            acc[6 + c] += ca.fc[3 * g + c];
        }
    }
    const double s9 = block_sum256<9>(acc, red);
    if (threadIdx.x < 9) sums[threadIdx.x] = s9;
    // several chains: each chain's centre of mass, in bead order
    if (M > 1)
        for (int ch = threadIdx.x; ch < M; ch += 256) {
            double cm[3] = {0, 0, 0};
            for (int k = 0; k < n; ++k) {
                const uint64_t g = bx.bead_off + (uint64_t)ch * n + k;
                for (int c = 0; c < 3; ++c) cm[c] += ca.x[3 * g + c];
            }
            for (int c = 0; c < 3; ++c) ccom[3 * ch + c] = cm[c] / n;
        }
    __syncthreads();
    double s = 0.0;
    for (int b = threadIdx.x; b < N; b += 256) {
        const uint64_t g = bx.bead_off + b;
        for (int c = 0; c < 3; ++c) {
            const double d = ca.x[3 * g + c] - (M > 1 ? ccom[3 * (b / n) + c] : sums[c] / N);
            s += d * d;
        }
    }
    double s1[1] = {s};
    const double sg = block_sum256<1>(s1, red1);
    if (threadIdx.x == 0) {
        double* o = out + (uint64_t)blockIdx.x * NCHAIN;
        for (int k = 0; k < 9; ++k) o[k] = sums[k];
        o[10] = sg;
        double e2 = 0.0;
        for (int ch = 0; ch < M; ++ch) {
            const uint64_t g0 = bx.bead_off + (uint64_t)ch * n, g1 = g0 + n - 1;
            for (int c = 0; c < 3; ++c) {
                const double d = ca.x[3 * g1 + c] - ca.x[3 * g0 + c];
                e2 += d * d;
            }
        }
        o[9] = e2;
    }
}

// --------------------------------------------------------------- launchers
static ChainArgs chain_args(const LaunchCtx& c)
{
    return ChainArgs{c.x, c.v, c.f, c.fc, c.nl_cnt, c.nl_idx, c.nl_x0, c.nl_cap, c.imp, c.touched,
                     c.touched_cnt, c.touch_cap, c.nl_rebuilds, c.vhist, c.hist_len, c.total_beads, c.tape,
                     c.tape_x0, c.tape_vo, c.tape_fo,
                     c.defer_on ? c.defer : nullptr, c.dclaim, c.defer_list, c.defer_cap, c.ovf, c.ovf_cap, c.ovm};
}

template <typename R, int W, bool PERSIST, int BT = 256>
static void launch_collide_v(const LaunchCtx& c, const void* A, void* B, int fixed_box, uint32_t tile0,
                             uint32_t n_tiles, uint32_t s_off)
{
    constexpr uint32_t M = BT / 256;
    const uint32_t groups = (n_tiles + M - 1) / M;
    const uint32_t grid = PERSIST ? std::min<uint32_t>(groups, (uint32_t)(c.n_cu * W)) : groups;
    hipLaunchKernelGGL((k_collide<R, W, PERSIST, BT>), dim3(grid), dim3(BT), 0, c.stream, c.boxes,
                       (const CollideConst<R>*)c.ccs, c.tile_box, fixed_box, tile0, n_tiles, (const R*)A, (R*)B,
                       c.ctrl, s_off, c.defer_on ? (const uint32_t*)c.defer : nullptr);
}

template <typename R>
hipError_t launch_collide(const LaunchCtx& c, const void* A, void* B, int fixed_box, uint32_t tile0,
                          uint32_t n_tiles, uint32_t s_off)
{
    if (n_tiles == 0) return hipSuccess;
    switch (c.collide_variant) {
    case 0: launch_collide_v<R, 4, false>(c, A, B, fixed_box, tile0, n_tiles, s_off); break;
    case 1: launch_collide_v<R, 5, false>(c, A, B, fixed_box, tile0, n_tiles, s_off); break;
    case 2: launch_collide_v<R, 6, false>(c, A, B, fixed_box, tile0, n_tiles, s_off); break;
    case 3: launch_collide_v<R, 7, false>(c, A, B, fixed_box, tile0, n_tiles, s_off); break;
    case 4: launch_collide_v<R, 8, false>(c, A, B, fixed_box, tile0, n_tiles, s_off); break;
    case 5: launch_collide_v<R, 4, true>(c, A, B, fixed_box, tile0, n_tiles, s_off); break;
    case 6: launch_collide_v<R, 5, true>(c, A, B, fixed_box, tile0, n_tiles, s_off); break;
    case 7: launch_collide_v<R, 6, true>(c, A, B, fixed_box, tile0, n_tiles, s_off); break;
    case 8: launch_collide_v<R, 7, true>(c, A, B, fixed_box, tile0, n_tiles, s_off); break;
    case 9: launch_collide_v<R, 8, true>(c, A, B, fixed_box, tile0, n_tiles, s_off); break;
    case 10: launch_collide_v<R, 4, false, 512>(c, A, B, fixed_box, tile0, n_tiles, s_off); break;
    case 11: launch_collide_v<R, 6, false, 512>(c, A, B, fixed_box, tile0, n_tiles, s_off); break;
    default: launch_collide_v<R, 4, false, 1024>(c, A, B, fixed_box, tile0, n_tiles, s_off); break;
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_fixup(const LaunchCtx& c, const void* A, void* B, uint64_t bead0, uint64_t n_beads,
                        uint32_t s_off)
{
    if (n_beads == 0) return hipSuccess;
    if (c.touch_cap < FIX_LANES) return hipErrorInvalidValue;
    const uint32_t n = (uint32_t)(n_beads * (uint64_t)FIX_LANES);
    hipLaunchKernelGGL(k_fixup<R>, dim3((n + 255) / 256), dim3(256), 0, c.stream, c.boxes,
                       (const CollideConst<R>*)c.ccs, c.bead_box, bead0, n, chain_args(c), c.claim,
                       (const R*)A, (R*)B, c.ctrl, s_off, c.keep_imp, c.defer_on);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_collide_deferred(const LaunchCtx& c, const void* A, void* B, uint32_t s_off)
{
    if (!c.defer_on || c.defer_cap == 0) return hipErrorInvalidValue;
    // a grid of a few blocks per CU strides over the list (its length is
    // known on the device only)
    const uint32_t grid = std::min<uint32_t>((c.defer_cap + DSEG_PER_TILE - 1) / DSEG_PER_TILE, (uint32_t)(4 * c.n_cu));
    hipLaunchKernelGGL(k_collide_deferred<R>, dim3(grid), dim3(256), 0, c.stream, c.boxes,
                       (const CollideConst<R>*)c.ccs, c.tile_box, (const uint32_t*)c.defer_list, c.defer_cap, c.imp,
                       (const R*)A, (R*)B, c.ctrl, s_off);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_overflow(const LaunchCtx& c, const void* A, void* B, uint32_t s_off, uint32_t advance)
{
    if (!c.defer_on) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_overflow<R>, dim3(1), dim3(256), 0, c.stream, c.boxes, (const CollideConst<R>*)c.ccs,
                       c.bead_box, chain_args(c), c.claim, (const R*)A, (R*)B, c.ctrl, s_off, advance);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_collide_forced(const LaunchCtx& c, const void* A, void* B, int fixed_box, uint32_t tile0,
                                 uint32_t n_tiles, uint32_t s_off)
{
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_collide_forced<R>, dim3(n_tiles), dim3(256), 0, c.stream, c.boxes,
                       (const CollideConst<R>*)c.ccs, c.tile_box, fixed_box, tile0, c.imp, (const R*)A, (R*)B,
                       c.ctrl, s_off);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_couple(const LaunchCtx& c, const void* A, const int32_t* list, int n_list, int block,
                         uint32_t s_off)
{
    if (n_list == 0) return hipSuccess;
    if (block > 256) return hipErrorInvalidValue;   // larger chains take the one-workgroup-per-chain kernel
    hipLaunchKernelGGL((k_couple<R, 256>), dim3(n_list), dim3(block), 0, c.stream, c.boxes, list, (const R*)A,
                       chain_args(c), c.ctrl, s_off);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_couple_big(const LaunchCtx& c, const void* A, const int32_t* list, int n_list, int max_n,
                             uint32_t s_off, hipEvent_t after_table, const void* Aprev, int single_box,
                             uint32_t wait_head, int zero_head, int stamp_next)
{
    if (n_list == 0) return hipSuccess;
    if (c.nl_cap > NL_SLOTS || max_n > WG_MAXB || max_n <= 0) return hipErrorInvalidValue;
    if ((Aprev || wait_head || stamp_next) && (c.dense_max_tiles || !c.defer_on)) return hipErrorInvalidValue;
    if (wait_head && (Aprev || after_table)) return hipErrorInvalidValue;
    const ChainArgs ca = chain_args(c);
    if (c.dense_max_tiles)
        hipLaunchKernelGGL(k_node_field<R>, dim3(c.dense_max_tiles, n_list), dim3(256), 0, c.stream, c.boxes, list,
                           (const R*)A, (R*)c.field);
    if (!wait_head)
        hipLaunchKernelGGL(k_near_nodes<R>, dim3((max_n * NEAR + 255) / 256, n_list), dim3(256), 0, c.stream,
                           c.boxes, list, (R*)A, ca, (R*)c.near_u, c.near_c, (const R*)c.field, c.ctrl, s_off,
                           (const CollideConst<R>*)c.ccs, c.bead_box, c.claim, (const R*)Aprev,
                           n_list == 1 && single_box >= 0 ? single_box : -1,
                           n_list == 1 && single_box >= 0 ? c.boxes_host[single_box] : BoxDev{}, zero_head);
    if (after_table) {
        const hipError_t e = hipEventRecord(after_table, c.stream);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_chain_wg<R>, dim3(n_list), dim3(WG_MAXB), 0, c.stream, c.boxes, list, (const R*)A, ca,
                       (const R*)c.near_u, (const int4*)c.near_c, c.sub_rec, c.ctrl, s_off, c.bead_box,
                       (Aprev || wait_head) ? 1 : 0, wait_head, stamp_next);
    if (c.big_sparse)
        hipLaunchKernelGGL(k_spread, dim3((max_n * 8 + 255) / 256, n_list), dim3(256), 0, c.stream, c.boxes, list,
                           ca, (const double*)c.sub_rec, c.ctrl, s_off);
    if (c.defer_on && c.big_sparse)
        hipLaunchKernelGGL(k_defer_list, dim3((max_n * NEAR + 255) / 256, n_list), dim3(256), 0, c.stream, c.boxes,
                           list, ca, (const int4*)c.near_c, c.ctrl, s_off);
    if (c.dense_max_tiles) {
        hipLaunchKernelGGL(k_bin_runs, dim3(n_list), dim3(WG_MAXB), 0, c.stream, c.boxes, list, ca,
                           (const double*)c.sub_rec, c.bin_start, c.slot_of);
        hipLaunchKernelGGL(k_run_impulse, dim3((max_n * 8 + 255) / 256, n_list), dim3(256), 0, c.stream, c.boxes,
                           list, ca, (const double*)c.sub_rec, (const uint32_t*)c.slot_of, c.runimp, c.ctrl);
        hipLaunchKernelGGL(k_gather_imp, dim3(c.dense_max_tiles, n_list), dim3(256), 0, c.stream, c.boxes, list, ca,
                           (const uint32_t*)c.bin_start, (const unsigned long long*)c.runimp);
    }
    return hipGetLastError();
}

template <typename R, int W>
static void launch_collide_headed_w(const LaunchCtx& c, const void* A, void* B, uint32_t n_tiles, uint32_t s_off,
                                    const int32_t* list, int n_list, int max_n, const void* Aprev, int single_box)
{
    const uint32_t head_x = (uint32_t)((max_n * NEAR + 255) / 256);
    const uint32_t n_head = head_blocks(n_list, max_n);
    hipLaunchKernelGGL((k_collide_headed<R, W>), dim3(n_head + n_tiles), dim3(256), 0, c.stream, c.boxes,
                       (const CollideConst<R>*)c.ccs, c.tile_box, (R*)A, (R*)B, c.ctrl, s_off,
                       (const uint32_t*)c.defer, n_head, head_x, list, chain_args(c), (R*)c.near_u, c.near_c,
                       c.bead_box, c.claim, (const R*)Aprev, n_list == 1 && single_box >= 0 ? single_box : -1,
                       n_list == 1 && single_box >= 0 ? c.boxes_host[single_box] : BoxDev{});
}

template <typename R>
hipError_t launch_collide_headed(const LaunchCtx& c, const void* A, void* B, uint32_t n_tiles, uint32_t s_off,
                                 const int32_t* list, int n_list, int max_n, const void* Aprev, int single_box)
{
    static_assert(NEAR == NEAR_ITEMS, "one table size");
    if (n_list == 0 || n_tiles == 0 || !Aprev || !c.defer_on || c.dense_max_tiles) return hipErrorInvalidValue;
    if (max_n > WG_MAXB || max_n <= 0) return hipErrorInvalidValue;
    // the node-table code caps the occupancy at 5 waves per SIMD, so the
    // launch shape keeps only the autotuned cap of 4
    if (c.collide_variant == 0)
        launch_collide_headed_w<R, 4>(c, A, B, n_tiles, s_off, list, n_list, max_n, Aprev, single_box);
    else
        launch_collide_headed_w<R, 5>(c, A, B, n_tiles, s_off, list, n_list, max_n, Aprev, single_box);
    return hipGetLastError();
}

hipError_t launch_init_forces(const LaunchCtx& c, const int32_t* list, int n_list, int block)
{
    if (n_list == 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_forces, dim3(n_list), dim3(block), 0, c.stream, c.boxes, list, c.x, c.f, c.ctrl);
    return hipGetLastError();
}

hipError_t launch_advance(const LaunchCtx& c, uint32_t n)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, c.stream, c.ctrl, n);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_stats(const LaunchCtx& c, const void* A, uint32_t max_recs, double* part, double* mid,
                        double* out)
{
    // every box's population array under 4 GiB: 32-bit offsets
    bool o32 = true;
    for (int b = 0; b < c.n_boxes; ++b)
        o32 = o32 && pop_elems_of((uint64_t)c.boxes_host[b].L * c.boxes_host[b].L * c.boxes_host[b].L) * sizeof(R) <
                         ((uint64_t)1 << 32);
    if (o32)
        hipLaunchKernelGGL((k_stats<R, true>), dim3(max_recs, c.n_boxes), dim3(256), 0, c.stream, c.boxes, (const R*)A,
                           part);
    else
        hipLaunchKernelGGL((k_stats<R, false>), dim3(max_recs, c.n_boxes), dim3(256), 0, c.stream, c.boxes,
                           (const R*)A, part);
    hipLaunchKernelGGL(k_stats_mid, dim3(STAT_CHUNKS, c.n_boxes), dim3(256), 0, c.stream, c.boxes, part, mid);
    hipLaunchKernelGGL(k_stats_final, dim3(c.n_boxes), dim3(64), 0, c.stream, mid, out);
    return hipGetLastError();
}

hipError_t launch_chain_obs(const LaunchCtx& c, double* out)
{
    hipLaunchKernelGGL(k_chain_obs, dim3(c.n_boxes), dim3(256), 0, c.stream, c.boxes, chain_args(c), out);
    return hipGetLastError();
}


// =================================================================== adjoint
// Reverse sweep of one LB step for the gradient of a loss of the bead
// velocities with respect to (omega_shear, omega_bulk, zeta).  The forward
// state of the step (pre-collision populations in the stored pull layout, the
// node impulses, the substep tape of the chain) comes from replaying the
// window segment; noise words are regenerated from Philox.  Adjoints are FP64.
//   lam_n[i * nodes + node]   adjoint of the pre-collision population n_i
//   lam_dp[c * nodes + node]  adjoint of the lattice impulse handed to a node

// VJP of one node's collision: given lam_o = dJ/d(post-collision d*), return
// lam_d = dJ/d(pre-collision d), lam_f = dJ/d(impulse), and the contributions
// to dJ/d(omega_s), dJ/d(omega_b).
__device__ __forceinline__ void collide_vjp(const double d[19], const double f[3], const CollideConst<double>& cc,
                                            uint32_t node, uint32_t step, uint32_t k0, uint32_t k1,
                                            const double lam_o[19], double lam_d[19], double lam_f[3],
                                            double& g_ws, double& g_wb)
{
    double m[19];
    to_modes<double>(d, m);
    const double rho = cc.rho0 + m[0], irho = 1.0 / rho;
    const double u[3] = {(m[1] + 0.5 * f[0]) * irho, (m[2] + 0.5 * f[1]) * irho, (m[3] + 0.5 * f[2]) * irho};
    const double e[10] = {0, 0, 0, 0, rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]),
                          rho * (2 * u[0] * u[0] - u[1] * u[1] - u[2] * u[2]), rho * (u[1] * u[1] - u[2] * u[2]),
                          rho * u[0] * u[1], rho * u[1] * u[2], rho * u[0] * u[2]};
    const double uf[3] = {u[0] * f[0], u[1] * f[1], u[2] * f[2]};
    const double sv[10] = {0, 0, 0, 0, 2 * (uf[0] + uf[1] + uf[2]), 2 * (2 * uf[0] - uf[1] - uf[2]), 2 * (uf[1] - uf[2]),
                           u[0] * f[1] + u[1] * f[0], u[1] * f[2] + u[2] * f[1], u[0] * f[2] + u[2] * f[0]};
    double r[19];
#pragma unroll
    for (int k = 0; k < 19; ++k) r[k] = 0.0;
    const double a = cc.therm > 0 ? sqrt(cc.mu * rho) : 0.0;
    if (cc.therm > 0) {
        const U4 w0 = philox10(U4{node, step, 0u, 0u}, k0, k1), w1 = philox10(U4{node, step, 0u, 1u}, k0, k1);
        r[4] = unit_noise<double>(w0.x); r[5] = unit_noise<double>(w0.y); r[6] = unit_noise<double>(w0.z);
        r[7] = unit_noise<double>(w0.w); r[8] = unit_noise<double>(w1.x); r[9] = unit_noise<double>(w1.y);
        if (cc.therm > 1) {
            const U4 w2 = philox10(U4{node, step, 0u, 2u}, k0, k1), w3 = philox10(U4{node, step, 0u, 3u}, k0, k1);
            r[10] = unit_noise<double>(w1.z); r[11] = unit_noise<double>(w1.w);
            r[12] = unit_noise<double>(w2.x); r[13] = unit_noise<double>(w2.y); r[14] = unit_noise<double>(w2.z);
            r[15] = unit_noise<double>(w2.w); r[16] = unit_noise<double>(w3.x); r[17] = unit_noise<double>(w3.y);
            r[18] = unit_noise<double>(w3.z);
        }
    }
    // d* = w_i sum_k e_ki M_k  ->  lam_M = E (w o lam_o)
    double wl[19], lM[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) wl[i] = wv(i) * lam_o[i];
    to_modes<double>(wl, lM);
    double lm[19];
#pragma unroll
    for (int k = 0; k < 19; ++k) lm[k] = 0.0;
    double lu[3] = {0, 0, 0}, lrho = 0.0, la = 0.0, lgs = 0.0, lgb = 0.0;
    lam_f[0] = lam_f[1] = lam_f[2] = 0.0;
    lm[0] += lM[0];
#pragma unroll
    for (int c = 0; c < 3; ++c) { lm[1 + c] += 3.0 * lM[1 + c]; lam_f[c] += 3.0 * lM[1 + c]; }
    double le[10], ls[10];
#pragma unroll
    for (int k = 4; k <= 9; ++k) {
        const double gam = k == 4 ? cc.gb : cc.gs, h = k == 4 ? cc.hb : cc.hs;
        const double lP = lM[k] * inv_b<double>(k);
        lm[k] += gam * lP;
        le[k] = (1.0 - gam) * lP;
        ls[k] = h * lP;
        double lg = (m[k] - e[k]) * lP + 0.5 * sv[k] * lP;
        if (cc.therm > 0 && cc.q[k] > 0.0) lg += a * r[k] * (-gam * inv_b<double>(k) / cc.q[k]) * lM[k];
        la += cc.q[k] * r[k] * lM[k];
        if (k == 4) lgb += lg; else lgs += lg;
    }
#pragma unroll
    for (int k = 10; k < 19; ++k) {
        lm[k] += cc.gg * inv_b<double>(k) * lM[k];
        la += cc.q[k] * r[k] * lM[k];
    }
    // equilibrium stress modes e_k(rho, u)
    lrho += (le[4] * e[4] + le[5] * e[5] + le[6] * e[6] + le[7] * e[7] + le[8] * e[8] + le[9] * e[9]) * irho;
    lu[0] += rho * (2 * u[0] * le[4] + 4 * u[0] * le[5] + u[1] * le[7] + u[2] * le[9]);
    lu[1] += rho * (2 * u[1] * le[4] - 2 * u[1] * le[5] + 2 * u[1] * le[6] + u[0] * le[7] + u[2] * le[8]);
    lu[2] += rho * (2 * u[2] * le[4] - 2 * u[2] * le[5] - 2 * u[2] * le[6] + u[1] * le[8] + u[0] * le[9]);
    // source terms s_k(u, f)
    lu[0] += 2 * f[0] * ls[4] + 4 * f[0] * ls[5] + f[1] * ls[7] + f[2] * ls[9];
    lu[1] += 2 * f[1] * ls[4] - 2 * f[1] * ls[5] + 2 * f[1] * ls[6] + f[0] * ls[7] + f[2] * ls[8];
    lu[2] += 2 * f[2] * ls[4] - 2 * f[2] * ls[5] - 2 * f[2] * ls[6] + f[1] * ls[8] + f[0] * ls[9];
    lam_f[0] += 2 * u[0] * ls[4] + 4 * u[0] * ls[5] + u[1] * ls[7] + u[2] * ls[9];
    lam_f[1] += 2 * u[1] * ls[4] - 2 * u[1] * ls[5] + 2 * u[1] * ls[6] + u[0] * ls[7] + u[2] * ls[8];
    lam_f[2] += 2 * u[2] * ls[4] - 2 * u[2] * ls[5] - 2 * u[2] * ls[6] + u[1] * ls[8] + u[0] * ls[9];
    // a = sqrt(mu rho)
    if (a > 0.0) lrho += la * a * 0.5 * irho;
    // u = (j + f/2) / rho
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lm[1 + c] += lu[c] * irho;
        lam_f[c] += 0.5 * lu[c] * irho;
    }
    lrho -= (u[0] * lu[0] + u[1] * lu[1] + u[2] * lu[2]) * irho;
    lm[0] += lrho;
    // m = E d  ->  lam_d = E^T lam_m
    from_scaled_modes<double>(lm, lam_d);
#pragma unroll
    for (int i = 0; i < 19; ++i) lam_d[i] /= wv(i);
    // gamma = 1 - omega
    g_ws = -lgs;
    g_wb = -lgb;
}

// One thread per node: lam_d*(r) is gathered from lam_n_next at the nodes the
// populations stream to (r + c_i); the forward state is the replayed
// pre-collision state.  Writes lam_n_cur and lam_dp; adds the tile's rate
// gradient to gpart[tile][2].
template <typename R>
__global__ __launch_bounds__(256) void k_adj_collide(const BoxDev* __restrict__ boxes,
                                                     const CollideConst<double>* __restrict__ ccd,
                                                     const uint32_t* __restrict__ tile_box,
                                                     const R* __restrict__ P, const unsigned long long* __restrict__ imp,
                                                     const double* __restrict__ lam_next, double* __restrict__ lam_cur,
                                                     double* __restrict__ lam_dp, double* __restrict__ gpart,
                                                     uint64_t nodes, uint32_t step)
{
    __shared__ double red[2][256];
    const uint32_t tile = blockIdx.x;
    const int bi = (int)tile_box[tile];
    const BoxDev& bx = boxes[bi];
    const int L = bx.L;
    const uint32_t V = (uint32_t)L * L * L;
    const uint32_t r = (tile - bx.tile_begin) * 256u + threadIdx.x;
    double gws = 0.0, gwb = 0.0;
    if (r < V) {
        const Upwind up = upwind_of(r, L, bx.inv_L);
        R dr[19];
        gather_pre<R, false>(P + bx.pop_off, up, dr);
        double d[19], f[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < 19; ++i) d[i] = (double)dr[i];
        const uint64_t gn = bx.node_off + r;
        if (bx.N > 0)
#pragma unroll
            for (int c = 0; c < 3; ++c) f[c] = (double)(long long)imp[3 * gn + c] * IMP_INV_SCALE;
        // the population leaving r along c_i arrives at r + c_i
        uint32_t x, y;
        const uint32_t q = div_L(r, L, bx.inv_L, &x);
        const uint32_t z = div_L(q, L, bx.inv_L, &y);
        const uint32_t Xd[3] = {x == 0 ? L - 1 : x - 1, x, x + 1 == (uint32_t)L ? 0 : x + 1};
        const uint32_t Yd[3] = {y == 0 ? L - 1 : y - 1, y, y + 1 == (uint32_t)L ? 0 : y + 1};
        const uint32_t Zd[3] = {z == 0 ? L - 1 : z - 1, z, z + 1 == (uint32_t)L ? 0 : z + 1};
        double lo[19];
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const uint32_t dn = Xd[cxv(i) + 1] + (uint32_t)L * (Yd[cyv(i) + 1] + (uint32_t)L * Zd[czv(i) + 1]);
            lo[i] = lam_next[i * nodes + bx.node_off + dn];
        }
        double ld[19], lf[3];
        collide_vjp(d, f, ccd[bi], r, step, bx.seed, bx.box_id, lo, ld, lf, gws, gwb);
#pragma unroll
        for (int i = 0; i < 19; ++i) lam_cur[i * nodes + gn] = ld[i];
#pragma unroll
        for (int c = 0; c < 3; ++c) lam_dp[c * nodes + gn] = lf[c];
    }
    red[0][threadIdx.x] = gws;
    red[1][threadIdx.x] = gwb;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        gpart[2 * (uint64_t)tile] += red[0][0];
        gpart[2 * (uint64_t)tile + 1] += red[1][0];
    }
}

// densities of the eight stencil nodes over the T lanes of one bead, as
// stencil_shared splits the corners: lane l sums corners l, l + T8, ... (NK
// of them, T8 = 8 / NK), then the lanes exchange the sums
template <typename R, int NK>
__device__ __forceinline__ void adj_densities(const R* __restrict__ a, const int i0[3], int L, double rho0,
                                              int lane, int T, double rho_k[8])
{
    constexpr int T8 = 8 / NK;
    const int k0 = lane & (T8 - 1);
    R dn[NK][19];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const int kk = k0 + k * T8;
        const int ix = i0[0] + (kk & 1), iy = i0[1] + ((kk >> 1) & 1), iz = i0[2] + ((kk >> 2) & 1);
        const Upwind up((uint32_t)(ix >= L ? ix - L : ix), (uint32_t)(iy >= L ? iy - L : iy),
                        (uint32_t)(iz >= L ? iz - L : iz), (uint32_t)L);
        gather_pre<R, false>(a, up, dn[k]);
    }
    double own[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        double rho = 0.0;
        for (int i = 0; i < 19; ++i) rho += (double)dn[k][i];
        own[k] = rho + rho0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) rho_k[k] = __shfl(own[k / T8], k % T8, T);
}

// add dJ/dv(end of step) and reverse the chain's substeps of one LB step; one
// workgroup per chain (at most 256 beads), thread per bead.
struct AdjChainArgs {
    const double* x0; const double* v0; const double* f0;   // bead state at the step start (replayed)
    const double* tape;                                     // [substep][total beads][TAPE_REC]
    const double* dj;                                       // dJ/dv at the step end [total beads][3]
    double* lx; double* lv; double* lf;                     // bead adjoints, in: step end, out: step start
    double* lam_n;                                          // pre-collision population adjoint (accumulated)
    const double* lam_dp;
    double* gz;                                             // per box dJ/dzeta
    uint64_t nodes, total_beads;
};

__device__ __forceinline__ void pair_kernel(const double d[3], double g, double gp, const double v[3], double out[3])
{
    // (g I + 2 g' d d^T) v
    const double dv = 2.0 * gp * (d[0] * v[0] + d[1] * v[1] + d[2] * v[2]);
    out[0] += g * v[0] + dv * d[0];
    out[1] += g * v[1] + dv * d[1];
    out[2] += g * v[2] + dv * d[2];
}

// Reverse sweep of one LB step's substeps for chains of at most 256 beads.
// Thread layout as in the forward kernel: T lanes per bead (T a function of
// N only), bead b = tid / T.  All lanes of a bead carry identical copies of
// the bead's adjoint; the repulsive-LJ pairs of the force Hessian are split
// over the lanes (partners j = lane mod T) and combined by a butterfly, which
// gives every lane the same bits, and every lane adds the two bonds' terms;
// the lanes share the stencil's density gathers; lane 0 writes and performs
// the atomics.
template <typename R>
__global__ __launch_bounds__(256) void k_adj_couple(const BoxDev* __restrict__ boxes,
                                                    const int32_t* __restrict__ couple_list, const R* __restrict__ P,
                                                    AdjChainArgs aa, uint32_t step)
{
    __shared__ double xs[3 * 256], lF[3 * 256], red[256];
    const int bi = couple_list[blockIdx.x];
    const BoxDev bx = boxes[bi];   // a copy: its fields stay in registers across the substeps
    const int N = bx.N, S = bx.substeps, L = bx.L;
    const int T = bx.couple_T;
    const int b = (int)threadIdx.x / T, lane = (int)threadIdx.x % T;
    const bool act = b < N;
    const bool writer = act && lane == 0;
    const uint64_t g = bx.bead_off + (uint64_t)(act ? b : 0);
    const ChainSpan sp = chain_span(bx, act ? b : 0);
    const double dt = bx.dt, h = 0.5 * dt / bx.mass, tau = bx.tau_lb, Ld = (double)L, iL = bx.inv_L;
    const double eps24 = 24.0 * bx.eps, s6c = bx.sigsq * bx.sigsq * bx.sigsq, s12c = s6c * s6c;
    double lx[3] = {0, 0, 0}, lv[3] = {0, 0, 0}, lf[3] = {0, 0, 0};
    if (act)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lx[c] = aa.lx[3 * g + c]; lv[c] = aa.lv[3 * g + c] + aa.dj[3 * g + c]; lf[c] = aa.lf[3 * g + c];
        }
    double gz = 0.0;
    int cb[3] = {-1, -1, -1};
    double lcu[8][3];          // accumulated adjoint of the stencil's node velocities
    double rho_k[8];
    uint32_t cnode[8];
    double cuk[8][3];
    double la[8][3];           // tau * lam_dp at the stencil's nodes
    bool have = false;
    const R* pb = P + bx.pop_off;
    auto flush = [&]() __attribute__((always_inline)) {   // node velocity adjoint -> population adjoint at the stencil nodes
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double ir = 1.0 / (rho_k[k] * tau);
            const double ul[3] = {cuk[k][0] * tau, cuk[k][1] * tau, cuk[k][2] * tau};
            for (int i = 0; i < 19; ++i) {
                const double cc = (double)cxv(i) * lcu[k][0] + (double)cyv(i) * lcu[k][1] + (double)czv(i) * lcu[k][2];
                const double lsum = lcu[k][0] * ul[0] + lcu[k][1] * ul[1] + lcu[k][2] * ul[2];
                atomicAdd(&aa.lam_n[i * aa.nodes + bx.node_off + cnode[k]], (cc - lsum) * ir);
            }
        }
    };
    // tape record of substep s, loaded one substep ahead
    double nx1[3] = {0, 0, 0}, nv1[3] = {0, 0, 0}, nfc[3] = {0, 0, 0}, nfr[3] = {0, 0, 0}, ni0[3] = {0, 0, 0};
    auto load_rec = [&](int s) __attribute__((always_inline)) {
        const double* tq = aa.tape + ((uint64_t)s * aa.total_beads + g) * TAPE_REC;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            nx1[c] = tq[c]; nv1[c] = tq[3 + c]; nfc[c] = tq[6 + c]; ni0[c] = tq[9 + c]; nfr[c] = tq[12 + c];
        }
    };
    if (act) load_rec(S - 1);
    for (int s = S - 1; s >= 0; --s) {
        const double* tp = aa.tape + ((uint64_t)s * aa.total_beads + g) * TAPE_REC;
        double x1[3], v1[3], fc[3], fr[3];
        int i0[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) { x1[c] = nx1[c]; v1[c] = nv1[c]; fc[c] = nfc[c]; i0[c] = (int)ni0[c]; fr[c] = nfr[c]; }
        if (act && s > 0) load_rec(s - 1);
        // v' = v1 + f' h and f' = F_c + fc
        double lft[3], lv1[3], lfc[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) { lft[c] = lf[c] + h * lv[c]; lv1[c] = lv[c]; lfc[c] = lft[c]; }
        if (writer) {
            xs[3 * b] = x1[0]; xs[3 * b + 1] = x1[1]; xs[3 * b + 2] = x1[2];
            lF[3 * b] = lft[0]; lF[3 * b + 1] = lft[1]; lF[3 * b + 2] = lft[2];
        }
        __syncthreads();
        double lx1[3] = {lx[0], lx[1], lx[2]};
        if (act) {
            // stencil of this substep
            if (i0[0] != cb[0] || i0[1] != cb[1] || i0[2] != cb[2]) {
                if (have && lane == 0) flush();
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int ix = i0[0] + (k & 1), iy = i0[1] + ((k >> 1) & 1), iz = i0[2] + ((k >> 2) & 1);
                    const uint32_t nx = ix >= L ? ix - L : ix, ny = iy >= L ? iy - L : iy, nz = iz >= L ? iz - L : iz;
                    cnode[k] = nx + (uint32_t)L * (ny + (uint32_t)L * nz);
                }
                // the densities of the 8 nodes, gathered by the bead's lanes
                // together (T is uniform over the workgroup)
                if (T >= 8) adj_densities<R, 1>(pb, i0, L, bx.rho0, lane, T, rho_k);
                else if (T == 4) adj_densities<R, 2>(pb, i0, L, bx.rho0, lane, T, rho_k);
                else if (T == 2) adj_densities<R, 4>(pb, i0, L, bx.rho0, lane, T, rho_k);
                else {
                    // one lane per bead: all eight, in batches whose loads are
                    // issued before any is summed
                    constexpr int NB = sizeof(R) == 4 ? 8 : 4;
#pragma unroll
                    for (int k0 = 0; k0 < 8; k0 += NB) {
                        R dn[NB][19];
#pragma unroll
                        for (int kk = 0; kk < NB; ++kk) {
                            const int k = k0 + kk;
                            const int ix = i0[0] + (k & 1), iy = i0[1] + ((k >> 1) & 1), iz = i0[2] + ((k >> 2) & 1);
                            const Upwind up((uint32_t)(ix >= L ? ix - L : ix), (uint32_t)(iy >= L ? iy - L : iy),
                                            (uint32_t)(iz >= L ? iz - L : iz), (uint32_t)L);
                            gather_pre<R, false>(pb, up, dn[kk]);
                        }
#pragma unroll
                        for (int kk = 0; kk < NB; ++kk) {
                            double rho = 0.0;
                            for (int i = 0; i < 19; ++i) rho += (double)dn[kk][i];
                            rho_k[k0 + kk] = rho + bx.rho0;
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const uint64_t gn = bx.node_off + cnode[k];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        cuk[k][c] = tp[15 + 3 * k + c];
                        lcu[k][c] = 0.0;
                        la[k][c] = tau * aa.lam_dp[c * aa.nodes + gn];
                    }
                }
                cb[0] = i0[0]; cb[1] = i0[1]; cb[2] = i0[2];
                have = true;
            }
            double wt[8], ub[3] = {0, 0, 0};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                wt[k] = ((k & 1) ? fr[0] : 1.0 - fr[0]) * (((k >> 1) & 1) ? fr[1] : 1.0 - fr[1]) *
                        (((k >> 2) & 1) ? fr[2] : 1.0 - fr[2]);
                ub[0] += wt[k] * cuk[k][0]; ub[1] += wt[k] * cuk[k][1]; ub[2] += wt[k] * cuk[k][2];
            }
            // impulse spread: acc_k -= w_k fc dt, handed over as tau * acc
            double lw[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const double la0 = la[k][0], la1 = la[k][1], la2 = la[k][2];
                lfc[0] -= dt * wt[k] * la0; lfc[1] -= dt * wt[k] * la1; lfc[2] -= dt * wt[k] * la2;
                lw[k] = -dt * (fc[0] * la0 + fc[1] * la1 + fc[2] * la2);
            }
            // fc = -zeta (v1 - u_b) + A(zeta) r
            const U4 w = philox10(U4{(uint32_t)b, step, (1u << 16) | (uint32_t)s, 0u}, bx.seed, bx.box_id);
            const double rn[3] = {unit_noise<double>(w.x), unit_noise<double>(w.y), unit_noise<double>(w.z)};
            double lub[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (bx.zeta > 0.0) gz += 0.5 * bx.bead_noise / bx.zeta * rn[c] * lfc[c];
                gz -= (v1[c] - ub[c]) * lfc[c];
                lv1[c] -= bx.zeta * lfc[c];
                lub[c] = bx.zeta * lfc[c];
            }
            // u_b = sum_k w_k cu_k
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                lw[k] += cuk[k][0] * lub[0] + cuk[k][1] * lub[1] + cuk[k][2] * lub[2];
                lcu[k][0] += wt[k] * lub[0]; lcu[k][1] += wt[k] * lub[1]; lcu[k][2] += wt[k] * lub[2];
            }
            // trilinear weights w_k(fractions of x1)
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const double g0 = (k & 1) ? fr[0] : 1.0 - fr[0], g1 = ((k >> 1) & 1) ? fr[1] : 1.0 - fr[1],
                             g2 = ((k >> 2) & 1) ? fr[2] : 1.0 - fr[2];
                lx1[0] += lw[k] * ((k & 1) ? 1.0 : -1.0) * g1 * g2;
                lx1[1] += lw[k] * (((k >> 1) & 1) ? 1.0 : -1.0) * g0 * g2;
                lx1[2] += lw[k] * (((k >> 2) & 1) ? 1.0 : -1.0) * g0 * g1;
            }
            // conservative forces at x1: lam_x1_b += sum_j K_bj (lam_F_b - lam_F_j).
            // The repulsive LJ pairs: this lane's share of the partners, four
            // at a time (their terms are computed side by side, then added in
            // ascending j), summed over the lanes
            double lp[3] = {0, 0, 0};
            for (int j0 = lane; j0 < N; j0 += 4 * T) {
                double d[4][3], dl[4][3], gw[4], gpw[4];
                bool hit[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int jj = j0 + u * T;
                    const int j = jj < N ? jj : b;   // past the end: the bead itself, masked
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        dl[u][c] = lft[c] - lF[3 * j + c];
                        d[u][c] = x1[c] - xs[3 * j + c];
                        d[u][c] -= Ld * rint(d[u][c] * iL);
                    }
                    const double q = d[u][0] * d[u][0] + d[u][1] * d[u][1] + d[u][2] * d[u][2];
                    hit[u] = j != b && q < bx.rc2;
                    const double iq = 1.0 / (hit[u] ? q : 1.0), iq4 = iq * iq * iq * iq, iq7 = iq4 * iq * iq * iq;
                    gw[u] = eps24 * (2.0 * s12c * iq7 - s6c * iq4);
                    gpw[u] = eps24 * (-14.0 * s12c * iq7 * iq + 4.0 * s6c * iq4 * iq);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (hit[u]) pair_kernel(d[u], gw[u], gpw[u], dl[u], lp);
            }
            for (int o = 1; o < T; o <<= 1) {
#pragma unroll
                for (int c = 0; c < 3; ++c) lp[c] += __shfl_xor(lp[c], o, T);
            }
            // the bonds (FENE) to b - 1 and b + 1, the same in every lane
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int j = side ? b + 1 : b - 1;
                if (j < sp.lo || j > sp.hi) continue;
                const double dl[3] = {lft[0] - lF[3 * j], lft[1] - lF[3 * j + 1], lft[2] - lF[3 * j + 2]};
                const double d[3] = {x1[0] - xs[3 * j], x1[1] - xs[3 * j + 1], x1[2] - xs[3 * j + 2]};
                const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                const double den = 1.0 - r2 * bx.inv_r0sq;
                const double gfe = -bx.k_fene / den;
                const double gpe = -bx.k_fene * bx.inv_r0sq / (den * den);
                pair_kernel(d, gfe, gpe, dl, lp);
            }
            lx1[0] += lp[0]; lx1[1] += lp[1]; lx1[2] += lp[2];
        }
        // x1 = x + v1 dt,  v1 = v + f h
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lv1[c] += dt * lx1[c];
            lx[c] = lx1[c];
            lv[c] = lv1[c];
            lf[c] = h * lv1[c];
        }
        __syncthreads();
    }
    if (writer) {
        if (have) flush();
#pragma unroll
        for (int c = 0; c < 3; ++c) { aa.lx[3 * g + c] = lx[c]; aa.lv[3 * g + c] = lv[c]; aa.lf[3 * g + c] = lf[c]; }
    }
    // dJ/dzeta of the box: one copy per bead, summed over a zero-padded array
    // (the block may hold fewer than 256 threads)
    for (int i = (int)threadIdx.x; i < 256; i += (int)blockDim.x) red[i] = 0.0;
    __syncthreads();
    if (writer) red[threadIdx.x] = gz;
    __syncthreads();
    for (int wdt = 128; wdt > 0; wdt >>= 1) {
        for (int i = (int)threadIdx.x; i < wdt; i += (int)blockDim.x) red[i] += red[i + wdt];
        __syncthreads();
    }
    if (threadIdx.x == 0) aa.gz[bi] += red[0];
}

template <typename R>
hipError_t launch_adj_collide(const LaunchCtx& c, const void* ccd, const void* P, const unsigned long long* imp,
                              const double* lam_next, double* lam_cur, double* lam_dp, double* gpart,
                              uint64_t nodes, uint32_t total_tiles, uint32_t step)
{
    hipLaunchKernelGGL(k_adj_collide<R>, dim3(total_tiles), dim3(256), 0, c.stream, c.boxes,
                       (const CollideConst<double>*)ccd, c.tile_box, (const R*)P, imp, lam_next, lam_cur, lam_dp,
                       gpart, nodes, step);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_adj_couple(const LaunchCtx& c, const int32_t* list, int n_list, int block, const void* P,
                             const AdjArgsHost& a, uint32_t step)
{
    if (n_list == 0) return hipSuccess;
    if (block < 64 || block > 256) return hipErrorInvalidValue;
    AdjChainArgs aa{a.x0, a.v0, a.f0, a.tape, a.dj, a.lx, a.lv, a.lf, a.lam_n, a.lam_dp, a.gz, a.nodes,
                    c.total_beads};
    hipLaunchKernelGGL(k_adj_couple<R>, dim3(n_list), dim3(block), 0, c.stream, c.boxes, list, (const R*)P, aa,
                       step);
    return hipGetLastError();
}

template hipError_t launch_adj_collide<float>(const LaunchCtx&, const void*, const void*, const unsigned long long*,
                                              const double*, double*, double*, double*, uint64_t, uint32_t, uint32_t);
template hipError_t launch_adj_collide<double>(const LaunchCtx&, const void*, const void*, const unsigned long long*,
                                               const double*, double*, double*, double*, uint64_t, uint32_t, uint32_t);
template hipError_t launch_adj_couple<float>(const LaunchCtx&, const int32_t*, int, int, const void*,
                                             const AdjArgsHost&, uint32_t);
template hipError_t launch_adj_couple<double>(const LaunchCtx&, const int32_t*, int, int, const void*,
                                              const AdjArgsHost&, uint32_t);

template hipError_t launch_collide<float>(const LaunchCtx&, const void*, void*, int, uint32_t, uint32_t, uint32_t);
template hipError_t launch_collide<double>(const LaunchCtx&, const void*, void*, int, uint32_t, uint32_t, uint32_t);
template hipError_t launch_fixup<float>(const LaunchCtx&, const void*, void*, uint64_t, uint64_t, uint32_t);
template hipError_t launch_fixup<double>(const LaunchCtx&, const void*, void*, uint64_t, uint64_t, uint32_t);
template hipError_t launch_collide_deferred<float>(const LaunchCtx&, const void*, void*, uint32_t);
template hipError_t launch_collide_deferred<double>(const LaunchCtx&, const void*, void*, uint32_t);
template hipError_t launch_overflow<float>(const LaunchCtx&, const void*, void*, uint32_t, uint32_t);
template hipError_t launch_overflow<double>(const LaunchCtx&, const void*, void*, uint32_t, uint32_t);
template hipError_t launch_collide_forced<float>(const LaunchCtx&, const void*, void*, int, uint32_t, uint32_t,
                                                 uint32_t);
template hipError_t launch_collide_forced<double>(const LaunchCtx&, const void*, void*, int, uint32_t, uint32_t,
                                                  uint32_t);
template hipError_t launch_couple<float>(const LaunchCtx&, const void*, const int32_t*, int, int, uint32_t);
template hipError_t launch_couple<double>(const LaunchCtx&, const void*, const int32_t*, int, int, uint32_t);
template hipError_t launch_couple_big<float>(const LaunchCtx&, const void*, const int32_t*, int, int, uint32_t,
                                            hipEvent_t, const void*, int, uint32_t, int, int);
template hipError_t launch_couple_big<double>(const LaunchCtx&, const void*, const int32_t*, int, int, uint32_t,
                                             hipEvent_t, const void*, int, uint32_t, int, int);
template hipError_t launch_collide_headed<float>(const LaunchCtx&, const void*, void*, uint32_t, uint32_t,
                                                 const int32_t*, int, int, const void*, int);
template hipError_t launch_collide_headed<double>(const LaunchCtx&, const void*, void*, uint32_t, uint32_t,
                                                  const int32_t*, int, int, const void*, int);
template hipError_t launch_stats<float>(const LaunchCtx&, const void*, uint32_t, double*, double*, double*);
template hipError_t launch_stats<double>(const LaunchCtx&, const void*, uint32_t, double*, double*, double*);

}  // namespace lbd
