/*
 * Oracle for the fluctuating D3Q19 lattice-Boltzmann step with a dissipatively
 * coupled bead-spring chain (Pham, Schiller, Prakash, Duenweg, arXiv:0903.5067).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, FP64 CPU statement
 * of what the GPU library computes.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may build, load or call it.  It shares
 * no code, header or table with the HIP library: the velocity set, the mode
 * basis, the Philox generator and every formula below are written out here on
 * their own.
 *
 * What each part follows:
 *   - LB equation (collide, then move n_i along c_i):   Sec. II.B, LB equation
 *   - second-order equilibrium n_i^eq(rho,u):           Sec. II.B, equilibrium eq.
 *   - D3Q19 velocities and weights, c_s^2 = 1/3:        Sec. II.B, text after eq.
 *   - thermalize every non-conserved mode:              Sec. II.B, last paragraphs
 *   - friction + Langevin force on the bead, momentum
 *     handed back to the surrounding fluid:             Sec. II.B, coupling paragraph
 *   - FENE and LJ (cut at 2^(1/6) sigma) potentials:    Sec. II.A, potentials
 *   - R_g^2 and R_e^2:                                  Sec. III.A, first equations
 *   - several chains in one box (semidilute solution):  Sec. III.C, Efficiency
 * Where the paper is silent (mode basis, noise law, forcing scheme, stencil
 * convention, MD integrator, units) the reading used is the one listed in the
 * design notes of this repository; each such place is marked "reading:" below.
 *
 * Canonical state: pre-collision populations n_i(r,t), FP64, plane-major
 * n[i*V + r] with r = x + L*(y + L*z), V = L^3; beads x, v (MD units),
 * f = total force of the last substep, fc = its coupling part (friction+noise).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

/* The step is written once as templates over the scalar type.  With double it
 * is the oracle; with D3 (a value and its derivatives with respect to the
 * three rates omega_shear, omega_bulk and zeta, forward-mode differentiation)
 * the same arithmetic yields the exact tangent of every quantity, used as the
 * oracle gradient of the adjoint window.  Integer decisions (stencil cell,
 * minimum image, LJ cut-off) are taken on values; their derivative is zero. */
struct D3 {
    double v;
    double d[3];
    D3() : v(0.0), d{0.0, 0.0, 0.0} {}
    D3(double x) : v(x), d{0.0, 0.0, 0.0} {}
};
static inline D3 operator+(const D3& a, const D3& b) { D3 r(a.v + b.v); for (int i = 0; i < 3; i++) r.d[i] = a.d[i] + b.d[i]; return r; }
static inline D3 operator-(const D3& a, const D3& b) { D3 r(a.v - b.v); for (int i = 0; i < 3; i++) r.d[i] = a.d[i] - b.d[i]; return r; }
static inline D3 operator-(const D3& a) { D3 r(-a.v); for (int i = 0; i < 3; i++) r.d[i] = -a.d[i]; return r; }
static inline D3 operator*(const D3& a, const D3& b) { D3 r(a.v * b.v); for (int i = 0; i < 3; i++) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
static inline D3 operator/(const D3& a, const D3& b)
{
    D3 r(a.v / b.v);
    for (int i = 0; i < 3; i++) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
    return r;
}
static inline D3 operator+(const D3& a, double b) { return a + D3(b); }
static inline D3 operator+(double a, const D3& b) { return D3(a) + b; }
static inline D3 operator-(const D3& a, double b) { return a - D3(b); }
static inline D3 operator-(double a, const D3& b) { return D3(a) - b; }
static inline D3 operator*(const D3& a, double b) { D3 r(a.v * b); for (int i = 0; i < 3; i++) r.d[i] = a.d[i] * b; return r; }
static inline D3 operator*(double a, const D3& b) { return b * a; }
static inline D3 operator/(const D3& a, double b) { return a / D3(b); }
static inline D3 operator/(double a, const D3& b) { return D3(a) / b; }
static inline D3& operator+=(D3& a, const D3& b) { a = a + b; return a; }
static inline D3& operator-=(D3& a, const D3& b) { a = a - b; return a; }
static inline D3& operator*=(D3& a, const D3& b) { a = a * b; return a; }
static inline D3& operator/=(D3& a, const D3& b) { a = a / b; return a; }
static inline D3 sqrt(const D3& a)
{
    D3 r(sqrt(a.v));
    for (int i = 0; i < 3; i++) r.d[i] = r.v > 0.0 ? a.d[i] / (2.0 * r.v) : 0.0;
    return r;
}
static inline double val(double a) { return a; }
static inline double val(const D3& a) { return a.v; }

/* the differentiated parameters, as scalars of the working type */
template <class T> struct Theta { T omega_s, omega_b, zeta; };

extern "C" {
void orc_tables(double* c, double* w, double* e, double* b);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_unit_noise(uint32_t word);
int orc_num_threads(void);
void orc_set_threads(int n);
}

typedef struct {
    int32_t L, N;
    double rho0, omega_s, omega_b, omega_g, kT;
    int32_t therm; /* 0 none, 1 stress modes only, 2 all non-conserved modes */
    double tau_lb, md_dt;
    int32_t md_substeps;
    double mass, zeta, k_fene, r0_fene, eps_wca, sigma_wca;
    uint32_t seed, box_id;
    int32_t chain_len; /* beads per chain; the N beads form N / chain_len chains of
                          consecutive indices; 0 = a single chain of N */
} orc_box;

extern "C" {
void orc_collide_stream(const orc_box* p, const double* nin, double* nout, const double* dp, uint32_t t);
void orc_collide_one(const orc_box* p, const double* n, const double* dp, uint32_t r, uint32_t t, double* nout);
void orc_initial_forces(const orc_box* p, const double* x, double* f);
void orc_couple(const orc_box* p, const double* n, double* x, double* v, double* f, double* fc, uint32_t t,
                double* dp);
void orc_run(const orc_box* p, double* n, double* x, double* v, double* f, double* fc, uint32_t t0,
             int32_t n_steps, double* vel_hist);
void orc_window_tangent(const orc_box* p, double* n, double* x, double* v, double* f, double* fc, uint32_t t0,
                        int32_t n_steps, double* vel_hist, double* dvel);
void orc_observables(const orc_box* p, const double* n, const double* x, const double* v, const double* fc,
                     double* out);
}

/* ---------------------------------------------------------------- D3Q19 --- */
/* rest, 6 nearest (|c|=1), 12 next-nearest (|c|=sqrt 2) neighbours; Sec. II.B */
static const int C[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {1, -1, 0}, {-1, 1, 0}, {-1, -1, 0},
    {1, 0, 1}, {1, 0, -1}, {-1, 0, 1}, {-1, 0, -1},
    {0, 1, 1}, {0, 1, -1}, {0, -1, 1}, {0, -1, -1}};

static double weight_of(int i)
{
    int c2 = C[i][0] * C[i][0] + C[i][1] * C[i][1] + C[i][2] * C[i][2];
    if (c2 == 0) return 1.0 / 3.0;
    if (c2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* reading: orthogonal mode basis of the Duenweg-Schiller-Ladd lineage the
 * paper cites for full thermalization.  e_k(c) as polynomials in c. */
static double mode_poly(int k, const int c[3])
{
    double cx = c[0], cy = c[1], cz = c[2];
    double c2 = cx * cx + cy * cy + cz * cz;
    switch (k) {
    case 0: return 1.0;
    case 1: return cx;
    case 2: return cy;
    case 3: return cz;
    case 4: return c2 - 1.0;
    case 5: return 3.0 * cx * cx - c2;
    case 6: return cy * cy - cz * cz;
    case 7: return cx * cy;
    case 8: return cy * cz;
    case 9: return cx * cz;
    case 10: return (3.0 * c2 - 5.0) * cx;
    case 11: return (3.0 * c2 - 5.0) * cy;
    case 12: return (3.0 * c2 - 5.0) * cz;
    case 13: return (cy * cy - cz * cz) * cx;
    case 14: return (cz * cz - cx * cx) * cy;
    case 15: return (cx * cx - cy * cy) * cz;
    case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    case 17: return (2.0 * c2 - 3.0) * (3.0 * cx * cx - c2);
    case 18: return (2.0 * c2 - 3.0) * (cy * cy - cz * cz);
    }
    return 0.0;
}

static double W[19], E[19][19], B[19];
static int tables_ready = 0;

static void build_tables(void)
{
    if (tables_ready) return;
    for (int i = 0; i < 19; i++) W[i] = weight_of(i);
    for (int k = 0; k < 19; k++) {
        B[k] = 0.0;
        for (int i = 0; i < 19; i++) {
            E[k][i] = mode_poly(k, C[i]);
            B[k] += W[i] * E[k][i] * E[k][i];
        }
    }
    tables_ready = 1;
}

void orc_tables(double* c, double* w, double* e, double* b)
{
    build_tables();
    for (int i = 0; i < 19; i++) {
        for (int a = 0; a < 3; a++) c[3 * i + a] = C[i][a];
        w[i] = W[i];
    }
    for (int k = 0; k < 19; k++) {
        b[k] = B[k];
        for (int i = 0; i < 19; i++) e[19 * k + i] = E[k][i];
    }
}

/* --------------------------------------------------------------- Philox --- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
 * multiplies and xors, the key bumped by the golden-ratio Weyl constants. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* reading: unit-variance uniform noise from the top 24 bits of a word,
 * r = sqrt(12) * (U - 1/2) with U = (v + 1/2) 2^-24, written as an odd
 * integer times 2^-25 so that it is exact before the sqrt(12) scaling. */
double orc_unit_noise(uint32_t word)
{
    int32_t v = (int32_t)(word >> 8);
    double k = (double)(2 * v - (1 << 24) + 1);
    return sqrt(12.0) * (k * 0x1p-25);
}

enum { PURPOSE_LB = 0, PURPOSE_BEAD = 1 };

/* noise word q (0..15) for LB node r at step t: counter (r, t, 0, q/4) */
static uint32_t lb_word(const orc_box* p, uint32_t r, uint32_t t, int q)
{
    uint32_t ctr[4] = {r, t, (uint32_t)PURPOSE_LB << 16, (uint32_t)(q / 4)};
    uint32_t key[2] = {p->seed, p->box_id};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[q % 4];
}

/* ------------------------------------------------------------- collision --- */
/* One node: populations n[19] (FP64, full n not deviations), lattice-unit
 * impulse dp[3] handed to the fluid this step, node index r, step t.
 * Output: post-collision populations nout[19]. */
template <class T>
static void collide_node(const orc_box* p, const Theta<T>& th, const T n[19], const T dp[3],
                         uint32_t r, uint32_t t, T nout[19])
{
    T m[19], ms[19];
    for (int k = 0; k < 19; k++) {
        m[k] = 0.0;
        for (int i = 0; i < 19; i++) m[k] += E[k][i] * n[i];
    }
    T rho = m[0];
    /* reading: second-order forcing; velocity shifted by half the impulse */
    T u[3];
    for (int a = 0; a < 3; a++) u[a] = (m[1 + a] + 0.5 * dp[a]) / rho;
    T u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];

    /* equilibrium stress modes: projections of the second-order n^eq */
    T meq[10];
    meq[4] = rho * u2;
    meq[5] = rho * (2.0 * u[0] * u[0] - u[1] * u[1] - u[2] * u[2]);
    meq[6] = rho * (u[1] * u[1] - u[2] * u[2]);
    meq[7] = rho * u[0] * u[1];
    meq[8] = rho * u[1] * u[2];
    meq[9] = rho * u[0] * u[2];
    /* projections of the source tensor u dp + dp u onto the stress modes */
    T src[10];
    src[4] = 2.0 * (u[0] * dp[0] + u[1] * dp[1] + u[2] * dp[2]);
    src[5] = 2.0 * (2.0 * u[0] * dp[0] - u[1] * dp[1] - u[2] * dp[2]);
    src[6] = 2.0 * (u[1] * dp[1] - u[2] * dp[2]);
    src[7] = u[0] * dp[1] + u[1] * dp[0];
    src[8] = u[1] * dp[2] + u[2] * dp[1];
    src[9] = u[0] * dp[2] + u[2] * dp[0];

    T gam[19];
    for (int k = 0; k < 19; k++) gam[k] = 0.0;
    gam[4] = 1.0 - th.omega_b;
    for (int k = 5; k <= 9; k++) gam[k] = 1.0 - th.omega_s;
    for (int k = 10; k <= 18; k++) gam[k] = 1.0 - p->omega_g;

    /* fluctuation amplitude: mu = kT / c_s^2 in lattice units,
     * kT_lat = kT * tau_lb^2 (lattice spacing 1, mass unit 1) */
    double kT_lat = p->kT * p->tau_lb * p->tau_lb;
    double mu = kT_lat * 3.0;
    int k_last = p->therm == 2 ? 18 : (p->therm == 1 ? 9 : 3);

    ms[0] = rho;
    for (int a = 0; a < 3; a++) ms[1 + a] = m[1 + a] + dp[a];
    for (int k = 4; k <= 9; k++)
        ms[k] = meq[k] + gam[k] * (m[k] - meq[k]) + 0.5 * (1.0 + gam[k]) * src[k];
    for (int k = 10; k <= 18; k++) ms[k] = gam[k] * m[k];
    for (int k = 4; k <= k_last; k++) {
        T sigma = sqrt(mu * rho * B[k] * (1.0 - gam[k] * gam[k]));
        ms[k] += sigma * orc_unit_noise(lb_word(p, r, t, k - 4));
    }
    for (int i = 0; i < 19; i++) {
        T s = 0.0;
        for (int k = 0; k < 19; k++) s += E[k][i] * ms[k] / B[k];
        nout[i] = W[i] * s;
    }
}

template <class T> static Theta<T> theta_of(const orc_box* p);
template <> Theta<double> theta_of<double>(const orc_box* p) { return {p->omega_s, p->omega_b, p->zeta}; }
template <> Theta<D3> theta_of<D3>(const orc_box* p)
{
    Theta<D3> th{D3(p->omega_s), D3(p->omega_b), D3(p->zeta)};
    th.omega_s.d[0] = 1.0;
    th.omega_b.d[1] = 1.0;
    th.zeta.d[2] = 1.0;
    return th;
}

static int wrap(int a, int L)
{
    a %= L;
    return a < 0 ? a + L : a;
}

/* collide every node with impulse field dp[3*V] (lattice units, NULL = 0),
 * then move each post-collision population to r + c_i (periodic). */
template <class T>
static void collide_stream(const orc_box* p, const Theta<T>& th, const T* nin, T* nout, const T* dp, uint32_t t)
{
    build_tables();
    const int L = p->L;
    const long V = (long)L * L * L;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < L; z++)
        for (int y = 0; y < L; y++)
            for (int x = 0; x < L; x++) {
                long r = x + (long)L * (y + (long)L * z);
                T n[19], ns[19], f[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < 19; i++) n[i] = nin[i * V + r];
                if (dp)
                    for (int a = 0; a < 3; a++) f[a] = dp[a * V + r];
                collide_node(p, th, n, f, (uint32_t)r, t, ns);
                for (int i = 0; i < 19; i++) {
                    int xd = wrap(x + C[i][0], L), yd = wrap(y + C[i][1], L),
                        zd = wrap(z + C[i][2], L);
                    nout[i * V + xd + (long)L * (yd + (long)L * zd)] = ns[i];
                }
            }
}

void orc_collide_stream(const orc_box* p, const double* nin, double* nout, const double* dp, uint32_t t)
{
    collide_stream<double>(p, theta_of<double>(p), nin, nout, dp, t);
}

/* single-node collision for tests (no streaming) */
void orc_collide_one(const orc_box* p, const double* n, const double* dp, uint32_t r,
                     uint32_t t, double* nout)
{
    build_tables();
    double f[3] = {0.0, 0.0, 0.0};
    if (dp) memcpy(f, dp, sizeof f);
    collide_node<double>(p, theta_of<double>(p), n, f, r, t, nout);
}

/* ------------------------------------------------------------ chain / MD --- */
/* beads per chain: a box holds N / chain_len chains (the semidilute solution
 * of M chains that Sec. III.C, Efficiency, discusses), a single chain otherwise */
static int chain_length(const orc_box* p) { return p->chain_len > 0 ? p->chain_len : p->N; }

/* force on bead b from bead j: FENE if bonded, i.e. neighbours along the same
 * chain (unwrapped separation), then the purely repulsive LJ with minimum
 * image between every pair; Sec. II.A.  Beads j are visited in ascending order
 * and the sum is taken in that order. */
template <class T>
static void conservative_force(const orc_box* p, const T* x, int b, T F[3])
{
    const double L = p->L;
    const double rc2 = pow(2.0, 1.0 / 3.0) * p->sigma_wca * p->sigma_wca;
    const int n = chain_length(p);
    F[0] = F[1] = F[2] = 0.0;
    for (int j = 0; j < p->N; j++) {
        if (j == b) continue;
        T d[3];
        if ((j == b - 1 || j == b + 1) && j / n == b / n) {
            for (int a = 0; a < 3; a++) d[a] = x[3 * b + a] - x[3 * j + a];
            T r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            /* -dV/dr along d for V = -(k R0^2/2) ln(1 - r^2/R0^2) */
            T g = -p->k_fene / (1.0 - r2 / (p->r0_fene * p->r0_fene));
            for (int a = 0; a < 3; a++) F[a] += g * d[a];
        }
        for (int a = 0; a < 3; a++) {
            T s = x[3 * b + a] - x[3 * j + a];
            d[a] = s - L * nearbyint(val(s) / L);
        }
        T r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (val(r2) < rc2) {
            /* -dV/dr along d for V = 4 eps [(s/r)^12 - (s/r)^6 + 1/4] */
            T s2 = p->sigma_wca * p->sigma_wca / r2;
            T s6 = s2 * s2 * s2;
            T g = 24.0 * p->eps_wca * s6 * (2.0 * s6 - 1.0) / r2;
            for (int a = 0; a < 3; a++) F[a] += g * d[a];
        }
    }
}

void orc_initial_forces(const orc_box* p, const double* x, double* f)
{
    for (int b = 0; b < p->N; b++) conservative_force<double>(p, x, b, f + 3 * b);
}

/* reading: nodes at integer coordinates; linear interpolation along each axis
 * between the two nearest planes of nodes, wrapped periodically. */
template <class T>
static void stencil(int L, const T x[3], long node[8], T wt[8])
{
    int i0[3];
    T fr[3];
    for (int a = 0; a < 3; a++) {
        T xt = x[a] - L * floor(val(x[a]) / L);
        double fl = floor(val(xt));
        fr[a] = xt - fl;
        i0[a] = wrap((int)fl, L);
    }
    for (int c = 0; c < 8; c++) {
        int d[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
        T w = 1.0;
        int idx[3];
        for (int a = 0; a < 3; a++) {
            w *= d[a] ? fr[a] : 1.0 - fr[a];
            idx[a] = wrap(i0[a] + d[a], L);
        }
        node[c] = idx[0] + (long)L * (idx[1] + (long)L * idx[2]);
        wt[c] = w;
    }
}

/* Velocity-Verlet substeps of the chain in a fluid velocity field frozen at
 * the pre-collision state of step t; the impulse taken from the beads by
 * friction and noise is handed to the nodes of each bead's stencil.
 * dp (3*V, lattice units) is overwritten. */
template <class T>
static void couple(const orc_box* p, const Theta<T>& th, const T* n, T* x, T* v, T* f, T* fc, uint32_t t,
                   T* dp)
{
    build_tables();
    const int L = p->L, N = p->N;
    const long V = (long)L * L * L;
    const double dt = p->md_dt, m = p->mass;
    /* frozen node velocities in MD units: u = (j / rho) / tau_lb */
    std::vector<T> u(3 * V);
    for (long r = 0; r < V; r++) {
        T rho = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < 19; i++) {
            T ni = n[i * V + r];
            rho += ni;
            for (int a = 0; a < 3; a++) j[a] += ni * (double)C[i][a];
        }
        for (int a = 0; a < 3; a++) u[a * V + r] = j[a] / rho / p->tau_lb;
    }
    for (long q = 0; q < 3 * V; q++) dp[q] = 0.0;
    const T noise_amp = sqrt(2.0 * p->kT * th.zeta / dt);
    std::vector<T> Fc(3 * (N > 0 ? N : 1));
    for (int s = 0; s < p->md_substeps; s++) {
        for (int b = 0; b < N; b++)
            for (int a = 0; a < 3; a++) {
                v[3 * b + a] += f[3 * b + a] / m * (0.5 * dt);
                x[3 * b + a] += v[3 * b + a] * dt;
            }
        for (int b = 0; b < N; b++) conservative_force<T>(p, x, b, &Fc[3 * b]);
        for (int b = 0; b < N; b++) {
            long node[8];
            T wt[8], ub[3] = {0.0, 0.0, 0.0};
            stencil<T>(L, x + 3 * b, node, wt);
            for (int c = 0; c < 8; c++)
                for (int a = 0; a < 3; a++) ub[a] += wt[c] * u[a * V + node[c]];
            uint32_t ctr[4] = {(uint32_t)b, t, ((uint32_t)PURPOSE_BEAD << 16) | (uint32_t)s, 0};
            uint32_t key[2] = {p->seed, p->box_id};
            uint32_t words[4];
            orc_philox4x32_10(ctr, key, words);
            for (int a = 0; a < 3; a++) {
                T ffr = -th.zeta * (v[3 * b + a] - ub[a]);
                T frn = noise_amp * orc_unit_noise(words[a]);
                fc[3 * b + a] = ffr + frn;
                f[3 * b + a] = Fc[3 * b + a] + fc[3 * b + a];
                v[3 * b + a] += f[3 * b + a] / m * (0.5 * dt);
            }
            for (int c = 0; c < 8; c++)
                for (int a = 0; a < 3; a++) dp[a * V + node[c]] -= wt[c] * fc[3 * b + a] * dt;
        }
    }
    /* MD impulse -> lattice units: p_lat = p_MD * tau_lb / (m_unit * a) */
    for (long q = 0; q < 3 * V; q++) dp[q] *= p->tau_lb;
}

void orc_couple(const orc_box* p, const double* n, double* x, double* v, double* f, double* fc, uint32_t t,
                double* dp)
{
    couple<double>(p, theta_of<double>(p), n, x, v, f, fc, t, dp);
}

/* n_steps full steps from step index t0: couple (if there are beads), then
 * collide+stream.  vel_hist (nullable) receives the bead velocities at the end
 * of each step, [n_steps][N][3]. */
template <class T>
static void run(const orc_box* p, const Theta<T>& th, T* n, T* x, T* v, T* f, T* fc, uint32_t t0,
                int32_t n_steps, T* vel_hist)
{
    build_tables();
    const long V = (long)p->L * p->L * p->L;
    std::vector<T> tmp(19 * V);
    std::vector<T> dp(p->N > 0 ? 3 * V : 0);
    for (int32_t s = 0; s < n_steps; s++) {
        uint32_t t = t0 + (uint32_t)s;
        if (p->N > 0) couple<T>(p, th, n, x, v, f, fc, t, dp.data());
        collide_stream<T>(p, th, n, tmp.data(), p->N > 0 ? dp.data() : nullptr, t);
        for (long q = 0; q < 19 * V; q++) n[q] = tmp[q];
        if (vel_hist)
            for (int q = 0; q < 3 * p->N; q++) vel_hist[(size_t)s * 3 * p->N + q] = v[q];
    }
}

void orc_run(const orc_box* p, double* n, double* x, double* v, double* f, double* fc, uint32_t t0,
             int32_t n_steps, double* vel_hist)
{
    run<double>(p, theta_of<double>(p), n, x, v, f, fc, t0, n_steps, vel_hist);
}

/* Forward-mode tangent of a window of n_steps steps from the given state (the
 * state itself does not depend on the rates): advances the state in place
 * exactly as orc_run does, fills vel_hist [n_steps][N][3] and its derivatives
 * dvel [n_steps][N][3][3] with respect to (omega_shear, omega_bulk, zeta). */
void orc_window_tangent(const orc_box* p, double* n, double* x, double* v, double* f, double* fc, uint32_t t0,
                        int32_t n_steps, double* vel_hist, double* dvel)
{
    const long V = (long)p->L * p->L * p->L;
    const int N = p->N;
    std::vector<D3> nd(n, n + 19 * V), xd(x, x + 3 * N), vd(v, v + 3 * N), fd(f, f + 3 * N),
        fcd(fc, fc + 3 * N), hd((size_t)n_steps * 3 * N);
    run<D3>(p, theta_of<D3>(p), nd.data(), xd.data(), vd.data(), fd.data(), fcd.data(), t0, n_steps, hd.data());
    for (long q = 0; q < 19 * V; q++) n[q] = nd[q].v;
    for (int q = 0; q < 3 * N; q++) { x[q] = xd[q].v; v[q] = vd[q].v; f[q] = fd[q].v; fc[q] = fcd[q].v; }
    for (size_t q = 0; q < (size_t)n_steps * 3 * N; q++) {
        vel_hist[q] = hd[q].v;
        for (int k = 0; k < 3; k++) dvel[3 * q + k] = hd[q].d[k];
    }
}

/* Observables, FP64, fixed summation order.  Layout of out[]:
 *  0 mass, 1-3 fluid momentum (lattice), 4-6 fluid momentum (MD),
 *  7-9 bead momentum, 10-12 conserved total (fluid + beads + dt/2 sum fc),
 *  13-15 centre of mass of all beads, 16 R_g^2 and 17 R_e^2 (each the mean over
 *  the box's chains), 18 count of n_i < 0,
 *  19-37 sum over nodes of (m_k - rho0 delta_k0)^2, k = 0..18. */
void orc_observables(const orc_box* p, const double* n, const double* x, const double* v,
                     const double* fc, double* out)
{
    build_tables();
    const long V = (long)p->L * p->L * p->L;
    const int N = p->N;
    memset(out, 0, sizeof(double) * 38);
    for (long r = 0; r < V; r++) {
        double m[19];
        for (int k = 0; k < 19; k++) {
            m[k] = 0.0;
            for (int i = 0; i < 19; i++) m[k] += E[k][i] * n[i * V + r];
        }
        out[0] += m[0];
        for (int a = 0; a < 3; a++) out[1 + a] += m[1 + a];
        for (int i = 0; i < 19; i++)
            if (n[i * V + r] < 0.0) out[18] += 1.0;
        for (int k = 0; k < 19; k++) {
            double d = k == 0 ? m[0] - p->rho0 : m[k];
            out[19 + k] += d * d;
        }
    }
    for (int a = 0; a < 3; a++) out[4 + a] = out[1 + a] / p->tau_lb;
    for (int b = 0; b < N; b++)
        for (int a = 0; a < 3; a++) out[7 + a] += p->mass * v[3 * b + a];
    for (int a = 0; a < 3; a++) {
        double s = 0.0;
        for (int b = 0; b < N; b++) s += fc[3 * b + a];
        out[10 + a] = out[4 + a] + out[7 + a] + 0.5 * p->md_dt * s;
    }
    if (N > 0) {
        for (int b = 0; b < N; b++)
            for (int a = 0; a < 3; a++) out[13 + a] += x[3 * b + a];
        for (int a = 0; a < 3; a++) out[13 + a] /= N;
        /* per chain, averaged over the chains of the box:
         * R_g^2 = (1 / 2n^2) sum_ij r_ij^2 (pair form, Sec. III.A) and
         * R_e^2 = (r_n - r_1)^2 */
        const int n = chain_length(p), M = N / n;
        for (int c = 0; c < M; c++) {
            const double* xc = x + 3 * (size_t)c * n;
            double s = 0.0;
            for (int i = 0; i < n; i++)
                for (int j = 0; j < n; j++)
                    for (int a = 0; a < 3; a++) {
                        double d = xc[3 * i + a] - xc[3 * j + a];
                        s += d * d;
                    }
            out[16] += s / (2.0 * n * (double)n);
            double e2 = 0.0;
            for (int a = 0; a < 3; a++) {
                double d = xc[3 * (n - 1) + a] - xc[a];
                e2 += d * d;
            }
            out[17] += e2;
        }
        out[16] /= M;
        out[17] /= M;
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the OpenMP loops from here on (n >= 1) */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
