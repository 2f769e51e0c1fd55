// Device-side building blocks of the fluctuating D3Q19 LB step (gfx950).
//
// Per-node collision in moment space (Sec. II.B: LB equation, second-order
// equilibrium, thermalization of the non-conserved modes), the Philox4x32-10
// counter-based generator (Salmon et al., SC'11) and the box descriptor the
// kernels read.  Populations are stored as deviations d_i = n_i - w_i rho0.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbd {

// ---------------------------------------------------------------- box table
// One entry per box; the host fills it once at init.  Rates are stored as
// gamma = 1 - omega.  mu = kT_lat / c_s^2 with kT_lat = kT * tau_lb^2.
struct BoxDev {
    int32_t L, N;
    uint32_t seed, box_id;
    uint64_t node_off;   // first global node index of the box (impulse-table keys)
    uint64_t pop_off;    // element offset of the box's first population tile
    uint64_t bead_off;   // first global bead index
    uint64_t field_off;  // dense boxes: first node of the box in the node-velocity field
    uint64_t bin_off;    // dense boxes: first entry of the box's run bins (L^3 + 1 entries)
    uint64_t item_off;   // dense boxes: first slot of the box's stencil runs (at most N x substeps)
    uint32_t tile_begin; // first collide tile of the box
    uint32_t n_tiles;
    int32_t therm;       // 0 none, 1 stress modes, 2 all non-conserved modes
    int32_t substeps;
    int32_t couple_T;    // lanes per bead on the one-workgroup coupling path (a function of N only)
    int32_t chain_len;   // beads per chain (> 0; N for a single chain)
    int32_t dense;       // 1: beads cover much of the box; its collide follows the coupling and
                         // takes the node impulses itself (no fix-up pass)
    uint32_t stat_off;   // first record of the box's observable partials (one per STAT_TPB tiles)
    double rho0, gam_b, gam_s, gam_g, mu;
    double tau_lb, dt, mass, zeta, k_fene, r0sq, eps, sigsq, rc2, bead_noise;
    double inv_L, inv_r0sq;
};

// Population storage of a box: its nodes fall into tiles of PTILE
// consecutive nodes (x fastest), and a tile holds its 19 planes one after
// another, PTILE values each.  A wavefront's 19 loads or stores then fall in
// one 76 KB block (FP32) instead of 19 planes a box volume apart.
constexpr uint32_t PTILE_LOG = 10;
constexpr uint32_t PTILE = 1u << PTILE_LOG;
__host__ __device__ __forceinline__ uint64_t pop_at(int i, uint32_t r)
{
    return ((uint64_t)(r >> PTILE_LOG) * 19u + (uint32_t)i) * PTILE + (r & (PTILE - 1u));
}
// elements of one box's populations in one buffer
__host__ __device__ __forceinline__ uint64_t pop_elems_of(uint64_t V)
{
    return (V + PTILE - 1) / PTILE * 19u * PTILE;
}

// control block in device memory: step index read by every kernel so that a
// captured graph can be replayed without re-recording arguments
struct Ctrl {
    uint32_t step;
    uint32_t health;
    uint32_t defer_cnt;     // collide tiles deferred this step (reset at the step's end)
    uint32_t ovf_cnt;       // impulses of this step outside the deferred tiles
    uint32_t ovf_flag[2];   // [t & 1]: the deferral stamp of step t if it listed any such impulse
    uint32_t head_done[2];  // [t & 1]: node-table workgroups of step t's collide that are done
    uint32_t head_fix[2];   // [t & 1]: those that have done their part of step t-1's overflow fix-up
};

// Deferral is decided per segment of DSEG consecutive nodes of a box (one
// wavefront of a 256-node collide tile): each segment has one stamp per step
// parity, at defer[2 * segment + (t & 1)].
constexpr uint32_t DSEG = 64;
constexpr uint32_t DSEG_PER_TILE = 256 / DSEG;

// Tag of step t in the per-segment deferral stamps: never 0 (the cleared value),
// so a tile is deferred in step t exactly when its stamp equals this.  Stamps
// repeat every 2^31 steps; restoring an earlier step count clears them.
__device__ __forceinline__ uint32_t defer_stamp(uint32_t t) { return t | 0x80000000u; }

enum : uint32_t {
    H_DENSITY = 1u << 0,   // rho <= 0 or NaN at a node
    H_MACH = 1u << 1,      // |u| > 0.3 (lattice units) or NaN
    H_FENE = 1u << 2,      // bond stretched to >= R0
    H_TABLE = 1u << 3,     // impulse table full
    H_FIXED = 1u << 4,     // impulse outside the fixed-point range
    H_NLIST = 1u << 5,     // neighbour list overflow
    H_SYNC = 1u << 6,      // a bounded wait for a concurrent kernel gave up
};

// fixed-point scale of the node impulse accumulator (lattice momentum units):
// resolution 2^-52, range +-2^11 per node (a lattice momentum of 1 per node
// is already far beyond the Mach limit)
constexpr double IMP_SCALE = 4503599627370496.0;          // 2^52
constexpr double IMP_INV_SCALE = 1.0 / 4503599627370496.0;
constexpr double IMP_MAX = 1024.0;                        // |impulse| bound per contribution

// ----------------------------------------------------------------- Philox
struct U4 { uint32_t x, y, z, w; };

__host__ __device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        U4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// top 24 bits of a word -> odd integer in (-2^24, 2^24); times sqrt(12) 2^-25
// gives a unit-variance uniform variate
__host__ __device__ __forceinline__ int32_t noise_int(uint32_t w) { return (int32_t)((w >> 8) << 1) - (1 << 24) + 1; }

template <typename R> struct NoiseScale;
constexpr double SQRT12 = 3.4641016151377544;   // correctly rounded sqrt(12)
template <> struct NoiseScale<float> { static constexpr float v = (float)(SQRT12 * 0x1p-25); };
template <> struct NoiseScale<double> { static constexpr double v = SQRT12 * 0x1p-25; };

template <typename R>
__host__ __device__ __forceinline__ R unit_noise(uint32_t w) { return (R)noise_int(w) * NoiseScale<R>::v; }

// ----------------------------------------------------------- D3Q19 layout
// i: 0 rest; 1,2 +-x; 3,4 +-y; 5,6 +-z; 7..10 xy (++,+-,-+,--);
// 11..14 xz (++,+-,-+,--); 15..18 yz (++,+-,-+,--)
__host__ __device__ constexpr int cxv(int i)
{
    return (i == 1 || i == 7 || i == 8 || i == 11 || i == 12) ? 1
         : (i == 2 || i == 9 || i == 10 || i == 13 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr int cyv(int i)
{
    return (i == 3 || i == 7 || i == 9 || i == 15 || i == 16) ? 1
         : (i == 4 || i == 8 || i == 10 || i == 17 || i == 18) ? -1 : 0;
}
__host__ __device__ constexpr int czv(int i)
{
    return (i == 5 || i == 11 || i == 13 || i == 15 || i == 17) ? 1
         : (i == 6 || i == 12 || i == 14 || i == 16 || i == 18) ? -1 : 0;
}
__host__ __device__ constexpr double wv(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

// ------------------------------------------------------------ transforms
// Forward transform to the 19 orthogonal modes (mass, momentum, bulk, five
// shear, nine ghost) with pair sums and differences; entries of the mode
// matrix are 0, +-1, +-2.
template <typename R>
__host__ __device__ __forceinline__ void to_modes(const R n[19], R m[19])
{
    R sx = n[1] + n[2], dx = n[1] - n[2];
    R sy = n[3] + n[4], dy = n[3] - n[4];
    R sz = n[5] + n[6], dz = n[5] - n[6];
    // xy quartet: a(+,+) b(+,-) c(-,+) d(-,-)
    R xy_ab = n[7] + n[8], xy_cd = n[9] + n[10], xy_ab_ = n[7] - n[8], xy_cd_ = n[9] - n[10];
    R s_xy = xy_ab + xy_cd, x_xy = xy_ab - xy_cd, y_xy = xy_ab_ + xy_cd_, p_xy = xy_ab_ - xy_cd_;
    R xz_ab = n[11] + n[12], xz_cd = n[13] + n[14], xz_ab_ = n[11] - n[12], xz_cd_ = n[13] - n[14];
    R s_xz = xz_ab + xz_cd, x_xz = xz_ab - xz_cd, z_xz = xz_ab_ + xz_cd_, p_xz = xz_ab_ - xz_cd_;
    R yz_ab = n[15] + n[16], yz_cd = n[17] + n[18], yz_ab_ = n[15] - n[16], yz_cd_ = n[17] - n[18];
    R s_yz = yz_ab + yz_cd, y_yz = yz_ab - yz_cd, z_yz = yz_ab_ + yz_cd_, p_yz = yz_ab_ - yz_cd_;

    R s1 = sx + sy + sz;
    R s2 = s_xy + s_xz + s_yz;
    m[0] = n[0] + s1 + s2;
    m[1] = dx + x_xy + x_xz;
    m[2] = dy + y_xy + y_yz;
    m[3] = dz + z_xz + z_yz;
    m[4] = s2 - n[0];
    m[5] = 2 * sx - sy - sz + s_xy + s_xz - 2 * s_yz;
    m[6] = sy - sz + s_xy - s_xz;
    m[7] = p_xy;
    m[8] = p_yz;
    m[9] = p_xz;
    m[10] = x_xy + x_xz - 2 * dx;
    m[11] = y_xy + y_yz - 2 * dy;
    m[12] = z_xz + z_yz - 2 * dz;
    m[13] = x_xy - x_xz;
    m[14] = y_yz - y_xy;
    m[15] = z_xz - z_yz;
    m[16] = n[0] - 2 * s1 + s2;
    m[17] = sy + sz - 2 * sx + s_xy + s_xz - 2 * s_yz;
    m[18] = sz - sy + s_xy - s_xz;
}

// Back transform n_i = w_i sum_k e_k(c_i) M_k with M_k = m_k / b_k already
// divided by the mode norms.
template <typename R>
__host__ __device__ __forceinline__ void from_scaled_modes(const R M[19], R n[19])
{
    const R w0 = (R)(1.0 / 3.0), w1 = (R)(1.0 / 18.0), w2 = (R)(1.0 / 36.0);
    n[0] = w0 * (M[0] - M[4] + M[16]);
    R ax = M[0] + 2 * M[5] - 2 * M[16] - 2 * M[17], bx = M[1] - 2 * M[10];
    R ay = M[0] - M[5] + M[6] - 2 * M[16] + M[17] - M[18], by = M[2] - 2 * M[11];
    R az = M[0] - M[5] - M[6] - 2 * M[16] + M[17] + M[18], bz = M[3] - 2 * M[12];
    n[1] = w1 * (ax + bx); n[2] = w1 * (ax - bx);
    n[3] = w1 * (ay + by); n[4] = w1 * (ay - by);
    n[5] = w1 * (az + bz); n[6] = w1 * (az - bz);
    R c0 = M[0] + M[4] + M[16];
    {   // xy
        R S = c0 + M[5] + M[6] + M[17] + M[18], X = M[1] + M[10] + M[13], Y = M[2] + M[11] - M[14], P = M[7];
        R sp = S + P, sm = S - P, xpy = X + Y, xmy = X - Y;
        n[7] = w2 * (sp + xpy); n[10] = w2 * (sp - xpy); n[8] = w2 * (sm + xmy); n[9] = w2 * (sm - xmy);
    }
    {   // xz
        R S = c0 + M[5] - M[6] + M[17] - M[18], X = M[1] + M[10] - M[13], Z = M[3] + M[12] + M[15], P = M[9];
        R sp = S + P, sm = S - P, xpz = X + Z, xmz = X - Z;
        n[11] = w2 * (sp + xpz); n[14] = w2 * (sp - xpz); n[12] = w2 * (sm + xmz); n[13] = w2 * (sm - xmz);
    }
    {   // yz
        R S = c0 - 2 * M[5] - 2 * M[17], Y = M[2] + M[11] + M[14], Z = M[3] + M[12] - M[15], P = M[8];
        R sp = S + P, sm = S - P, ypz = Y + Z, ymz = Y - Z;
        n[15] = w2 * (sp + ypz); n[18] = w2 * (sp - ypz); n[16] = w2 * (sm + ymz); n[17] = w2 * (sm - ymz);
    }
}

// Collision constants of one box in the compute precision, prepared on the
// host: gamma = 1 - omega per class, h = (1 + gamma)/2, and the noise factor
// q_k = sqrt((1 - gamma_k^2) / b_k), so that the noise added to m_k / b_k is
// sqrt(mu rho) q_k r_k  (variance of m_k: mu rho b_k (1 - gamma_k^2)).
template <typename R>
struct CollideConst {
    R rho0, gb, gs, gg, hb, hs, mu;
    R q[19];
    int therm;
};

// inverse mode norms 1/b_k, b_k = sum_i w_i e_k(c_i)^2
template <typename R>
__host__ __device__ __forceinline__ R inv_b(int k)
{
    constexpr double ib[19] = {1.0, 3.0, 3.0, 3.0, 1.5, 0.75, 2.25, 9.0, 9.0, 9.0,
                               1.5, 1.5, 1.5, 4.5, 4.5, 4.5, 0.5, 0.75, 2.25};
    return (R)ib[k];
}

// Collide one node.  d: deviations d_i = n_i - w_i rho0 (in), out: post-collision
// deviations; (fx,fy,fz): lattice-unit impulse handed to the node this step;
// node, step and the box key (k0,k1) select the noise words.
// Returns health bits.
template <typename R>
__host__ __device__ __forceinline__ uint32_t collide(const R d[19], R out[19], R fx, R fy, R fz,
                                            const CollideConst<R>& cc, uint32_t node, uint32_t step,
                                            uint32_t k0, uint32_t k1)
{
    R m[19];
    to_modes(d, m);
    const R rho = cc.rho0 + m[0];
    const R irho = (R)1 / rho;
    const R ux = (m[1] + (R)0.5 * fx) * irho;
    const R uy = (m[2] + (R)0.5 * fy) * irho;
    const R uz = (m[3] + (R)0.5 * fz) * irho;
    const R uxx = ux * ux, uyy = uy * uy, uzz = uz * uz;
    const R u2 = uxx + uyy + uzz;
    uint32_t health = 0;
    if (!(rho > (R)0)) health |= H_DENSITY;
    if (!(u2 <= (R)0.09)) health |= H_MACH;

    // equilibrium stress modes (projections of the second-order n^eq) and the
    // projections of the source tensor u f + f u
    const R e4 = rho * u2, e5 = rho * (2 * uxx - uyy - uzz), e6 = rho * (uyy - uzz);
    const R e7 = rho * ux * uy, e8 = rho * uy * uz, e9 = rho * ux * uz;
    const R ufx = ux * fx, ufy = uy * fy, ufz = uz * fz;
    const R s4 = 2 * (ufx + ufy + ufz), s5 = 2 * (2 * ufx - ufy - ufz), s6 = 2 * (ufy - ufz);
    const R s7 = ux * fy + uy * fx, s8 = uy * fz + uz * fy, s9 = ux * fz + uz * fx;

    R M[19];
    M[0] = m[0];
    M[1] = (m[1] + fx) * (R)3;
    M[2] = (m[2] + fy) * (R)3;
    M[3] = (m[3] + fz) * (R)3;
    M[4] = (e4 + cc.gb * (m[4] - e4) + cc.hb * s4) * inv_b<R>(4);
    M[5] = (e5 + cc.gs * (m[5] - e5) + cc.hs * s5) * inv_b<R>(5);
    M[6] = (e6 + cc.gs * (m[6] - e6) + cc.hs * s6) * inv_b<R>(6);
    M[7] = (e7 + cc.gs * (m[7] - e7) + cc.hs * s7) * inv_b<R>(7);
    M[8] = (e8 + cc.gs * (m[8] - e8) + cc.hs * s8) * inv_b<R>(8);
    M[9] = (e9 + cc.gs * (m[9] - e9) + cc.hs * s9) * inv_b<R>(9);
#pragma unroll
    for (int k = 10; k < 19; ++k) M[k] = cc.gg * m[k] * inv_b<R>(k);

    if (cc.therm > 0) {
        const R a = sqrt(cc.mu * rho);
        // words 0..5 -> modes 4..9 (stress), words 6..14 -> modes 10..18 (ghosts)
        const U4 w0 = philox10(U4{node, step, 0u, 0u}, k0, k1);
        const U4 w1 = philox10(U4{node, step, 0u, 1u}, k0, k1);
        M[4] += a * cc.q[4] * unit_noise<R>(w0.x);
        M[5] += a * cc.q[5] * unit_noise<R>(w0.y);
        M[6] += a * cc.q[6] * unit_noise<R>(w0.z);
        M[7] += a * cc.q[7] * unit_noise<R>(w0.w);
        M[8] += a * cc.q[8] * unit_noise<R>(w1.x);
        M[9] += a * cc.q[9] * unit_noise<R>(w1.y);
        if (cc.therm > 1) {
            const U4 w2 = philox10(U4{node, step, 0u, 2u}, k0, k1);
            const U4 w3 = philox10(U4{node, step, 0u, 3u}, k0, k1);
            M[10] += a * cc.q[10] * unit_noise<R>(w1.z);
            M[11] += a * cc.q[11] * unit_noise<R>(w1.w);
            M[12] += a * cc.q[12] * unit_noise<R>(w2.x);
            M[13] += a * cc.q[13] * unit_noise<R>(w2.y);
            M[14] += a * cc.q[14] * unit_noise<R>(w2.z);
            M[15] += a * cc.q[15] * unit_noise<R>(w2.w);
            M[16] += a * cc.q[16] * unit_noise<R>(w3.x);
            M[17] += a * cc.q[17] * unit_noise<R>(w3.y);
            M[18] += a * cc.q[18] * unit_noise<R>(w3.z);
        }
    }
    from_scaled_modes(M, out);
    return health;
}

}  // namespace lbd
