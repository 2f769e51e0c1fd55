// HIP kernels of the fluctuating D3Q19 LB step with a dissipatively coupled
// bead-spring chain, for gfx950 (MI355X).
//
//   k_couple      one workgroup per chain: velocity-Verlet substeps in the
//                 fluid velocity field frozen at the pre-collision state,
//                 trilinear interpolation, friction + Langevin force, and the
//                 impulse handed back to the stencil nodes (Sec. II.B,
//                 coupling paragraph; potentials of Sec. II.A)
//   k_collide     fused collide + push-stream of every node, no impulse
//                 (Sec. II.B, LB equation), thread per node, SoA planes
//   k_fixup       re-collides the few nodes that received an impulse and
//                 overwrites their streamed outputs
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

// -------------------------------------------------------------- collide
template <typename R>
__global__ __launch_bounds__(256) void k_collide(const BoxDev* __restrict__ boxes,
                                                 const CollideConst<R>* __restrict__ ccs,
                                                 const uint32_t* __restrict__ tile_box,
                                                 int fixed_box, uint32_t tile0,
                                                 const R* __restrict__ A, R* __restrict__ B,
                                                 Ctrl* __restrict__ ctrl, uint32_t s_off)
{
    const uint32_t tile = tile0 + blockIdx.x;
    const int bi = fixed_box >= 0 ? fixed_box : (int)tile_box[tile];
    const BoxDev& bx = boxes[bi];
    const int L = bx.L;
    const uint32_t V = (uint32_t)L * L * L;
    const uint32_t r = (tile - bx.tile_begin) * 256u + threadIdx.x;
    if (r >= V) return;
    const uint32_t t = ctrl->step + s_off;
    const CollideConst<R> cc = ccs[bi];
    const uint64_t ps = bx.ps;
    const R* a = A + bx.pop_off + r;
    R d[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) d[i] = a[i * ps];
    R o[19];
    uint32_t h = collide<R>(d, o, (R)0, (R)0, (R)0, cc, r, t, bx.seed, bx.box_id);
    uint32_t x, y, z;
    uint32_t q = div_L(r, L, bx.inv_L, &x);
    z = div_L(q, L, bx.inv_L, &y);
    const uint32_t xm = x == 0 ? L - 1 : x - 1, xp = x + 1 == (uint32_t)L ? 0 : x + 1;
    const uint32_t ym = y == 0 ? L - 1 : y - 1, yp = y + 1 == (uint32_t)L ? 0 : y + 1;
    const uint32_t zm = z == 0 ? L - 1 : z - 1, zp = z + 1 == (uint32_t)L ? 0 : z + 1;
    const uint32_t X[3] = {xm, x, xp};
    const uint32_t Y[3] = {ym * L, y * L, yp * L};
    const uint32_t LL = (uint32_t)L * L;
    const uint32_t Z[3] = {zm * LL, z * LL, zp * LL};
    R* b = B + bx.pop_off;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const uint32_t dst = X[cxv(i) + 1] + Y[cyv(i) + 1] + Z[czv(i) + 1];
        b[i * ps + dst] = o[i];
    }
    if (h) atomicOr(&ctrl->health, h);
}

// ---------------------------------------------------------------- fixup
// One thread per impulse-table slot of the launched boxes.  The slot's key is
// 1 + local node index (0 = empty); values are fixed-point impulses.
template <typename R>
__global__ __launch_bounds__(256) void k_fixup(const BoxDev* __restrict__ boxes, int n_boxes,
                                               const CollideConst<R>* __restrict__ ccs,
                                               const uint32_t* __restrict__ tab_off,
                                               uint32_t slot0, uint32_t n_slots, int fixed_box,
                                               uint32_t* __restrict__ keys,
                                               unsigned long long* __restrict__ vals,
                                               const R* __restrict__ A, R* __restrict__ B,
                                               Ctrl* __restrict__ ctrl, uint32_t s_off)
{
    const uint32_t sidx = blockIdx.x * 256u + threadIdx.x;
    if (sidx >= n_slots) return;
    const uint32_t slot = slot0 + sidx;
    const uint32_t key = keys[slot];
    if (key == 0) return;
    int bi = fixed_box;
    if (bi < 0) {   // last box whose table starts at or before the slot
        int lo = 0, hi = n_boxes - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (tab_off[mid] <= slot) lo = mid; else hi = mid - 1;
        }
        bi = lo;
    }
    const BoxDev& bx = boxes[bi];
    const uint32_t r = key - 1;
    const int L = bx.L;
    const uint32_t t = ctrl->step + s_off;
    const CollideConst<R> cc = ccs[bi];
    const uint64_t ps = bx.ps;
    const R* a = A + bx.pop_off + r;
    R d[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) d[i] = a[i * ps];
    R f[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        f[c] = (R)((double)(long long)vals[3 * (uint64_t)slot + c] * IMP_INV_SCALE);
        vals[3 * (uint64_t)slot + c] = 0ull;
    }
    keys[slot] = 0u;
    R o[19];
    uint32_t h = collide<R>(d, o, f[0], f[1], f[2], cc, r, t, bx.seed, bx.box_id);
    uint32_t x, y, z;
    uint32_t q = div_L(r, L, bx.inv_L, &x);
    z = div_L(q, L, bx.inv_L, &y);
    const uint32_t xm = x == 0 ? L - 1 : x - 1, xp = x + 1 == (uint32_t)L ? 0 : x + 1;
    const uint32_t ym = y == 0 ? L - 1 : y - 1, yp = y + 1 == (uint32_t)L ? 0 : y + 1;
    const uint32_t zm = z == 0 ? L - 1 : z - 1, zp = z + 1 == (uint32_t)L ? 0 : z + 1;
    const uint32_t X[3] = {xm, x, xp};
    const uint32_t Y[3] = {ym * L, y * L, yp * L};
    const uint32_t LL = (uint32_t)L * L;
    const uint32_t Z[3] = {zm * LL, z * LL, zp * LL};
    R* b = B + bx.pop_off;
#pragma unroll
    for (int i = 0; i < 19; ++i) b[i * ps + X[cxv(i) + 1] + Y[cyv(i) + 1] + Z[czv(i) + 1]] = o[i];
    if (h) atomicOr(&ctrl->health, h);
}

// --------------------------------------------------------------- couple
struct ChainArgs {
    double* x; double* v; double* f; double* fc;   // [total beads][3]
    int32_t* nl_cnt; int32_t* nl_idx; double* nl_x0; int nl_cap;
    uint32_t* keys; unsigned long long* vals; const uint32_t* tab_off; const uint32_t* tab_cap;
    double* vhist; int hist_len; uint64_t total_beads;
};

__device__ __forceinline__ uint32_t hash_node(uint32_t k)
{
    k ^= k >> 16; k *= 0x7feb352dU; k ^= k >> 15; k *= 0x846ca68bU; k ^= k >> 16;
    return k;
}

// add a lattice-unit impulse (3 components) to local node r of the box's table
__device__ __forceinline__ uint32_t table_add(uint32_t* keys, unsigned long long* vals, uint32_t off,
                                              uint32_t cap, uint32_t r, const double p[3])
{
    uint32_t hbits = 0;
    unsigned long long q[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double v = p[c];
        if (!(fabs(v) < IMP_MAX)) { hbits |= H_FIXED; v = v > 0 ? IMP_MAX : -IMP_MAX; if (v != v) v = 0; }
        q[c] = (unsigned long long)(long long)llrint(v * IMP_SCALE);
    }
    const uint32_t key = r + 1;
    uint32_t s = hash_node(key) & (cap - 1);
    for (uint32_t probe = 0; probe < cap; ++probe) {
        uint32_t prev = atomicCAS(&keys[off + s], 0u, key);
        if (prev == 0u || prev == key) {
#pragma unroll
            for (int c = 0; c < 3; ++c) atomicAdd(&vals[3 * (uint64_t)(off + s) + c], q[c]);
            return hbits;
        }
        s = (s + 1) & (cap - 1);
    }
    return hbits | H_TABLE;
}

template <typename R>
__device__ __forceinline__ void node_velocity(const R* __restrict__ a, uint64_t ps, uint32_t r, double rho0,
                                              double inv_tau, double u[3])
{
    double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const double di = (double)a[i * ps + r];
        rho += di;
        if (cxv(i)) jx += cxv(i) * di;
        if (cyv(i)) jy += cyv(i) * di;
        if (czv(i)) jz += czv(i) * di;
    }
    rho += rho0;
    u[0] = jx / rho * inv_tau;
    u[1] = jy / rho * inv_tau;
    u[2] = jz / rho * inv_tau;
}

constexpr int MAXB = 1024;
constexpr double NL_SKIN = 0.5;

// Conservative force on bead b (Sec. II.A): FENE to the bonded neighbours
// (unwrapped separations), purely repulsive LJ to every other bead within the
// cut-off (minimum image).  xs: positions of all beads of the chain (LDS).
// nl: ascending list of candidate partners (cnt >= 0) or NULL for all beads.
__device__ __forceinline__ uint32_t cons_force(const BoxDev& bx, int b, int N, const double x[3],
                                               const double* xs, int cnt, const int32_t* nl, double F[3])
{
    const double Ld = (double)bx.L;
    uint32_t hb = 0;
    F[0] = F[1] = F[2] = 0.0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int j = side ? b + 1 : b - 1;
        if (j < 0 || j >= N) continue;
        const double d0 = x[0] - xs[3 * j], d1 = x[1] - xs[3 * j + 1], d2 = x[2] - xs[3 * j + 2];
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        double den = 1.0 - r2 / bx.r0sq;
        if (!(den > 0.0)) { hb |= H_FENE; den = 1e-12; }
        const double gf = -bx.k_fene / den;
        F[0] += gf * d0; F[1] += gf * d1; F[2] += gf * d2;
    }
    const int nloop = cnt >= 0 ? cnt : N;
    for (int jj = 0; jj < nloop; ++jj) {
        const int j = cnt >= 0 ? nl[jj] : jj;
        if (j == b) continue;
        double d0 = x[0] - xs[3 * j], d1 = x[1] - xs[3 * j + 1], d2 = x[2] - xs[3 * j + 2];
        d0 -= Ld * rint(d0 / Ld); d1 -= Ld * rint(d1 / Ld); d2 -= Ld * rint(d2 / Ld);
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        if (r2 < bx.rc2) {
            const double s2 = bx.sigsq / r2;
            const double s6 = s2 * s2 * s2;
            const double gf = 24.0 * bx.eps * s6 * (2.0 * s6 - 1.0) / r2;
            F[0] += gf * d0; F[1] += gf * d1; F[2] += gf * d2;
        }
    }
    return hb;
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
        double F[3];
        uint32_t hb = cons_force(bx, b, N, x, xs, -1, nullptr, F);
        for (int c = 0; c < 3; ++c) fg[3 * g + c] = F[c];
        if (hb) atomicOr(&ctrl->health, hb);
    }
}

template <typename R>
__global__ __launch_bounds__(1024) void k_couple(const BoxDev* __restrict__ boxes,
                                                 const int32_t* __restrict__ couple_list,
                                                 const R* __restrict__ A, ChainArgs ca,
                                                 Ctrl* __restrict__ ctrl, uint32_t s_off)
{
    __shared__ double xs[3 * MAXB];
    const int bi = couple_list[blockIdx.x];
    const BoxDev& bx = boxes[bi];
    const int N = bx.N;
    const int b = threadIdx.x;
    const bool act = b < N;
    const uint64_t g = bx.bead_off + (uint64_t)(act ? b : 0);
    const uint32_t t = ctrl->step + s_off;
    const int L = bx.L;
    const double Ld = (double)L;
    const double dt = bx.dt, m = bx.mass, hdt_m = 0.5 * dt / m;
    const double inv_tau = 1.0 / bx.tau_lb;
    const R* a = A + bx.pop_off;
    const uint32_t toff = ca.tab_off[bi], tcap = ca.tab_cap[bi];
    const bool use_nl = N > 64;
    const double rl = sqrt(bx.rc2) + NL_SKIN;
    const double rl2 = rl * rl;

    double x[3] = {0, 0, 0}, v[3] = {0, 0, 0}, f[3] = {0, 0, 0}, fcl[3] = {0, 0, 0};
    if (act) {
#pragma unroll
        for (int c = 0; c < 3; ++c) { x[c] = ca.x[3 * g + c]; v[c] = ca.v[3 * g + c]; f[c] = ca.f[3 * g + c]; }
    }
    int cb[3] = {-1, -1, -1};     // base cell of the cached stencil
    double cu[8][3];              // node velocities of the cached stencil (MD units)
    double acc[8][3];             // impulse accumulated on the cached stencil (MD units)
    uint32_t cnode[8];
    bool have_acc = false;
    uint32_t hbits = 0;

    for (int s = 0; s < bx.substeps; ++s) {
        if (act) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v[c] += f[c] * hdt_m;
                x[c] += v[c] * dt;
                xs[3 * b + c] = x[c];
            }
        }
        bool rebuild = false;
        if (use_nl && act) {
            const int cnt = ca.nl_cnt[g];
            const double dx0 = x[0] - ca.nl_x0[3 * g], dy0 = x[1] - ca.nl_x0[3 * g + 1], dz0 = x[2] - ca.nl_x0[3 * g + 2];
            rebuild = cnt == -2 || dx0 * dx0 + dy0 * dy0 + dz0 * dz0 > 0.25 * NL_SKIN * NL_SKIN;
        }
        rebuild = __syncthreads_or(rebuild);
        if (use_nl && rebuild && act) {
            int cnt = 0;
            for (int j = 0; j < N; ++j) {
                if (j == b) continue;
                double d0 = x[0] - xs[3 * j], d1 = x[1] - xs[3 * j + 1], d2 = x[2] - xs[3 * j + 2];
                d0 -= Ld * rint(d0 / Ld); d1 -= Ld * rint(d1 / Ld); d2 -= Ld * rint(d2 / Ld);
                if (d0 * d0 + d1 * d1 + d2 * d2 < rl2) {
                    if (cnt < ca.nl_cap) ca.nl_idx[g * ca.nl_cap + cnt] = j;
                    ++cnt;
                }
            }
            ca.nl_cnt[g] = cnt > ca.nl_cap ? -1 : cnt;   // -1: overflow, use the full loop
#pragma unroll
            for (int c = 0; c < 3; ++c) ca.nl_x0[3 * g + c] = x[c];
        }
        if (act) {
            double F[3];
            const int cnt = use_nl ? ca.nl_cnt[g] : -1;
            hbits |= cons_force(bx, b, N, x, xs, cnt, cnt >= 0 ? ca.nl_idx + g * ca.nl_cap : nullptr, F);
            // stencil of the bead: nodes at integer coordinates, periodic
            int i0[3];
            double fr[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double xt = x[c] - Ld * floor(x[c] / Ld);
                const double fl = floor(xt);
                fr[c] = xt - fl;
                int ii = (int)fl;
                if (ii >= L) ii -= L;
                if (ii < 0) ii += L;
                i0[c] = ii;
            }
            if (i0[0] != cb[0] || i0[1] != cb[1] || i0[2] != cb[2]) {
                if (have_acc) {
                    for (int k = 0; k < 8; ++k) {
                        const double p[3] = {acc[k][0] * bx.tau_lb, acc[k][1] * bx.tau_lb, acc[k][2] * bx.tau_lb};
                        hbits |= table_add(ca.keys, ca.vals, toff, tcap, cnode[k], p);
                    }
                }
                for (int k = 0; k < 8; ++k) {
                    const int ix = i0[0] + (k & 1), iy = i0[1] + ((k >> 1) & 1), iz = i0[2] + ((k >> 2) & 1);
                    const uint32_t rr = (uint32_t)(ix >= L ? ix - L : ix) +
                                        (uint32_t)L * ((uint32_t)(iy >= L ? iy - L : iy) +
                                                       (uint32_t)L * (uint32_t)(iz >= L ? iz - L : iz));
                    cnode[k] = rr;
                    node_velocity<R>(a, bx.ps, rr, bx.rho0, inv_tau, cu[k]);
                    acc[k][0] = acc[k][1] = acc[k][2] = 0.0;
                }
                cb[0] = i0[0]; cb[1] = i0[1]; cb[2] = i0[2];
                have_acc = true;
            }
            double wt[8], ub[3] = {0, 0, 0};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                wt[k] = ((k & 1) ? fr[0] : 1.0 - fr[0]) * (((k >> 1) & 1) ? fr[1] : 1.0 - fr[1]) *
                        (((k >> 2) & 1) ? fr[2] : 1.0 - fr[2]);
                ub[0] += wt[k] * cu[k][0]; ub[1] += wt[k] * cu[k][1]; ub[2] += wt[k] * cu[k][2];
            }
            const U4 w = philox10(U4{(uint32_t)b, t, (1u << 16) | (uint32_t)s, 0u}, bx.seed, bx.box_id);
            const uint32_t ws[3] = {w.x, w.y, w.z};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double ffr = -bx.zeta * (v[c] - ub[c]);
                const double frn = bx.bead_noise * unit_noise<double>(ws[c]);
                fcl[c] = ffr + frn;
                f[c] = F[c] + fcl[c];
                v[c] += f[c] * hdt_m;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                acc[k][0] -= wt[k] * fcl[0] * dt;
                acc[k][1] -= wt[k] * fcl[1] * dt;
                acc[k][2] -= wt[k] * fcl[2] * dt;
            }
        }
        __syncthreads();
    }
    if (act) {
        if (have_acc) {
            for (int k = 0; k < 8; ++k) {
                const double p[3] = {acc[k][0] * bx.tau_lb, acc[k][1] * bx.tau_lb, acc[k][2] * bx.tau_lb};
                hbits |= table_add(ca.keys, ca.vals, toff, tcap, cnode[k], p);
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ca.x[3 * g + c] = x[c]; ca.v[3 * g + c] = v[c]; ca.f[3 * g + c] = f[c]; ca.fc[3 * g + c] = fcl[c];
        }
        if (ca.vhist) {
            double* hv = ca.vhist + ((uint64_t)(t % (uint32_t)ca.hist_len) * ca.total_beads + g) * 3;
            hv[0] = v[0]; hv[1] = v[1]; hv[2] = v[2];
        }
        if (hbits) atomicOr(&ctrl->health, hbits);
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
constexpr int NSTAT = 24;

template <typename R>
__global__ __launch_bounds__(256) void k_stats(const BoxDev* __restrict__ boxes,
                                               const uint32_t* __restrict__ tile_box,
                                               const R* __restrict__ A, double* __restrict__ part)
{
    __shared__ double red[NSTAT][256];
    const uint32_t tile = blockIdx.x;
    const int bi = (int)tile_box[tile];
    const BoxDev& bx = boxes[bi];
    const uint32_t V = (uint32_t)bx.L * bx.L * bx.L;
    const uint32_t r = (tile - bx.tile_begin) * 256u + threadIdx.x;
    double acc[NSTAT];
#pragma unroll
    for (int k = 0; k < NSTAT; ++k) acc[k] = 0.0;
    if (r < V) {
        const R* a = A + bx.pop_off + r;
        double d[19], m[19];
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            d[i] = (double)a[i * bx.ps];
            if (wv(i) * bx.rho0 + d[i] < 0.0) acc[4] += 1.0;
        }
        to_modes<double>(d, m);
        acc[0] = m[0]; acc[1] = m[1]; acc[2] = m[2]; acc[3] = m[3];
#pragma unroll
        for (int k = 0; k < 19; ++k) acc[5 + k] = m[k] * m[k];
    }
#pragma unroll
    for (int k = 0; k < NSTAT; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < NSTAT; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < NSTAT) part[(uint64_t)tile * NSTAT + threadIdx.x] = red[threadIdx.x][0];
}

// one block per box: reduce the box's tile records in a fixed order
__global__ __launch_bounds__(256) void k_stats_final(const BoxDev* __restrict__ boxes,
                                                     const double* __restrict__ part, double* __restrict__ out)
{
    __shared__ double red[NSTAT][256];
    const BoxDev& bx = boxes[blockIdx.x];
    double acc[NSTAT];
    for (int k = 0; k < NSTAT; ++k) acc[k] = 0.0;
    for (uint32_t tt = threadIdx.x; tt < bx.n_tiles; tt += 256)
        for (int k = 0; k < NSTAT; ++k) acc[k] += part[(uint64_t)(bx.tile_begin + tt) * NSTAT + k];
    for (int k = 0; k < NSTAT; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < NSTAT; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < NSTAT) out[(uint64_t)blockIdx.x * NSTAT + threadIdx.x] = red[threadIdx.x][0];
}

// one block per box: chain sums.  Record: [0..2] sum x, [3..5] sum m v,
// [6..8] sum fc, [9] R_e^2, then after the second pass [10] sum |x - com|^2.
constexpr int NCHAIN = 11;

__global__ __launch_bounds__(256) void k_chain_obs(const BoxDev* __restrict__ boxes, ChainArgs ca,
                                                   double* __restrict__ out)
{
    __shared__ double red[9][256];
    __shared__ double sums[9];
    const BoxDev& bx = boxes[blockIdx.x];
    const int N = bx.N;
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
    for (int k = 0; k < 9; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 9; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 9) sums[threadIdx.x] = red[threadIdx.x][0];
    __syncthreads();
    double s = 0.0;
    for (int b = threadIdx.x; b < N; b += 256) {
        const uint64_t g = bx.bead_off + b;
        for (int c = 0; c < 3; ++c) {
            const double d = ca.x[3 * g + c] - sums[c] / N;
            s += d * d;
        }
    }
    red[0][threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[0][threadIdx.x] += red[0][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* o = out + (uint64_t)blockIdx.x * NCHAIN;
        for (int k = 0; k < 9; ++k) o[k] = sums[k];
        o[10] = red[0][0];
        double e2 = 0.0;
        if (N > 0) {
            const uint64_t g0 = bx.bead_off, g1 = bx.bead_off + N - 1;
            for (int c = 0; c < 3; ++c) {
                const double d = ca.x[3 * g1 + c] - ca.x[3 * g0 + c];
                e2 += d * d;
            }
        }
        o[9] = e2;
    }
}

// --------------------------------------------------------------- launchers
template <typename R>
hipError_t launch_collide(const LaunchCtx& c, const void* A, void* B, int fixed_box, uint32_t tile0,
                          uint32_t n_tiles, uint32_t s_off)
{
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_collide<R>, dim3(n_tiles), dim3(256), 0, c.stream, c.boxes,
                       (const CollideConst<R>*)c.ccs, c.tile_box, fixed_box, tile0, (const R*)A, (R*)B,
                       c.ctrl, s_off);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_fixup(const LaunchCtx& c, const void* A, void* B, int fixed_box, uint32_t slot0,
                        uint32_t n_slots, uint32_t s_off)
{
    if (n_slots == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fixup<R>, dim3((n_slots + 255) / 256), dim3(256), 0, c.stream, c.boxes, c.n_boxes,
                       (const CollideConst<R>*)c.ccs, c.tab_off, slot0, n_slots, fixed_box, c.keys, c.vals,
                       (const R*)A, (R*)B, c.ctrl, s_off);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_couple(const LaunchCtx& c, const void* A, const int32_t* list, int n_list, int block,
                         uint32_t s_off)
{
    if (n_list == 0) return hipSuccess;
    ChainArgs ca{c.x, c.v, c.f, c.fc, c.nl_cnt, c.nl_idx, c.nl_x0, c.nl_cap, c.keys, c.vals,
                 c.tab_off, c.tab_cap, c.vhist, c.hist_len, c.total_beads};
    hipLaunchKernelGGL(k_couple<R>, dim3(n_list), dim3(block), 0, c.stream, c.boxes, list, (const R*)A, ca,
                       c.ctrl, s_off);
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
hipError_t launch_stats(const LaunchCtx& c, const void* A, uint32_t total_tiles, double* part, double* out)
{
    hipLaunchKernelGGL(k_stats<R>, dim3(total_tiles), dim3(256), 0, c.stream, c.boxes, c.tile_box, (const R*)A,
                       part);
    hipLaunchKernelGGL(k_stats_final, dim3(c.n_boxes), dim3(256), 0, c.stream, c.boxes, part, out);
    return hipGetLastError();
}

hipError_t launch_chain_obs(const LaunchCtx& c, double* out)
{
    ChainArgs ca{c.x, c.v, c.f, c.fc, c.nl_cnt, c.nl_idx, c.nl_x0, c.nl_cap, c.keys, c.vals,
                 c.tab_off, c.tab_cap, c.vhist, c.hist_len, c.total_beads};
    hipLaunchKernelGGL(k_chain_obs, dim3(c.n_boxes), dim3(256), 0, c.stream, c.boxes, ca, out);
    return hipGetLastError();
}

template hipError_t launch_collide<float>(const LaunchCtx&, const void*, void*, int, uint32_t, uint32_t, uint32_t);
template hipError_t launch_collide<double>(const LaunchCtx&, const void*, void*, int, uint32_t, uint32_t, uint32_t);
template hipError_t launch_fixup<float>(const LaunchCtx&, const void*, void*, int, uint32_t, uint32_t, uint32_t);
template hipError_t launch_fixup<double>(const LaunchCtx&, const void*, void*, int, uint32_t, uint32_t, uint32_t);
template hipError_t launch_couple<float>(const LaunchCtx&, const void*, const int32_t*, int, int, uint32_t);
template hipError_t launch_couple<double>(const LaunchCtx&, const void*, const int32_t*, int, int, uint32_t);
template hipError_t launch_stats<float>(const LaunchCtx&, const void*, uint32_t, double*, double*);
template hipError_t launch_stats<double>(const LaunchCtx&, const void*, uint32_t, double*, double*);

}  // namespace lbd
