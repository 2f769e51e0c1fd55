/*
 * lbmd.h -- C ABI of the MI355X (gfx950) library for the fluctuating D3Q19
 * lattice-Boltzmann solvent with a dissipatively coupled bead-spring chain
 * (Pham, Schiller, Prakash, Duenweg, arXiv:0903.5067).
 *
 * The problem these calls set up follows the paper's statement of it: one
 * chain of N beads joined by FENE springs, with the purely repulsive
 * Lennard-Jones potential between all beads (Sec. II.A, potentials), immersed
 * in a periodic cubic box of L^3 lattice sites of LB fluid (Sec. II.B LB
 * equation; Sec. II.E cubic box with periodic boundaries) with density rho0,
 * relaxation rates and temperature kT, coupled by friction zeta_bare and a
 * Langevin force whose momentum is taken from the fluid (Sec. II.B, coupling
 * paragraph), advanced in MD steps md_dt and LB steps tau_lb
 * (Sec. II.E, time steps), and observed through mass, momentum and the chain's
 * R_g^2 and R_e^2 (Sec. III.A).  Several independent boxes (the finite-size
 * study of Sec. II.E / Sec. III.C) can be advanced together.
 *
 * Units: the chain in Lennard-Jones units (sigma = m = eps = 1); lattice
 * spacing 1 sigma; the LB step tau_lb in LJ time; rho0 in m / sigma^3; kT in
 * eps.  Relaxation rates omega are per LB step, omega = 1 - gamma.
 *
 * Conventions
 *  - Every call returns lb_status; nothing aborts or throws across the ABI.
 *    lb_last_error() gives a message for the last failing call on a handle
 *    (or, with NULL, the last failure of lb_query_sizes / lb_init in the
 *    calling thread).
 *  - Ownership: d_state and d_scratch are device memory owned by the caller
 *    (for example torch tensors), sized by lb_query_sizes, aligned to 256
 *    bytes, and must outlive the handle.  The handle owns only host metadata,
 *    captured graphs and, if the caller passes stream == NULL, a stream it
 *    creates.  lb_free never frees caller memory.
 *  - Streams: all device work is enqueued on the stream given to lb_init
 *    (a hipStream_t passed as void*).  lb_couple and lb_step return without
 *    synchronising; numeric failures are recorded in a device health word and
 *    reported by the next lb_observables / lb_export_state as LB_ENUMERIC.
 *  - Host buffers (bead_x0, export/import buffers, lb_obs arrays) are plain
 *    host memory owned by the caller.
 */
#ifndef LBMD_H
#define LBMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb_handle lb_handle;

typedef enum {
    LB_OK = 0,
    LB_EINVAL = -1,    /* invalid argument or parameter set */
    LB_ENOMEM = -2,    /* caller buffer too small */
    LB_EDEVICE = -3,   /* a HIP runtime call failed */
    LB_ENUMERIC = -4,  /* device health word set (see LB_HEALTH_*) */
    LB_ESTATE = -5     /* call not valid in the handle's current state */
} lb_status;

typedef enum { LB_FP64 = 0, LB_FP32_DEV = 1 } lb_precision;
/* thermalization of the non-conserved modes (Sec. II.B): none, the six
 * stress modes only (the original scheme), or all fifteen */
typedef enum { LB_THERM_OFF = 0, LB_THERM_STRESS = 1, LB_THERM_ALL = 2 } lb_thermalize;

/* health bits reported in lb_obs.health */
#define LB_HEALTH_DENSITY 0x1u  /* rho <= 0 or NaN at some node */
#define LB_HEALTH_MACH 0x2u     /* |u| > 0.3 lattice units (or NaN) at some node */
#define LB_HEALTH_FENE 0x4u     /* a bond reached R0 */
#define LB_HEALTH_TABLE 0x8u    /* a node-impulse list overflowed (touched nodes, impulses outside deferred tiles) */
#define LB_HEALTH_FIXED 0x10u   /* node impulse outside the fixed-point range */
#define LB_HEALTH_SYNC 0x40u    /* a bounded wait of one kernel for a concurrent one gave up (results of the step invalid) */

/* One box.  An array of these is a batch of independent boxes. */
typedef struct {
    int32_t L;            /* sites per edge, 2 <= L <= 1625; cubic, periodic, spacing 1 */
    int32_t n_beads;      /* N, 0 <= N <= min(1024, L^3); 0 = pure fluid.  The
                             beads of a box form one chain, or chain_len-bead
                             chains (see chain_len) */
    double rho0;          /* fluid density, > 0 */
    double omega_shear;   /* shear-mode relaxation rate, in (0, 2) */
    double omega_bulk;    /* bulk-mode relaxation rate, in (0, 2) */
    double omega_ghost;   /* rate of the nine ghost modes, in (0, 2) */
    double kT;            /* temperature (eps), >= 0 */
    int32_t thermalize;   /* lb_thermalize */
    double tau_lb;        /* LB step in LJ time; must equal md_substeps * md_dt */
    double md_dt;         /* MD step, > 0 */
    int32_t md_substeps;  /* MD steps per LB step, >= 1 */
    double bead_mass;     /* > 0 */
    double zeta;          /* bare friction coefficient, >= 0 */
    double k_fene;        /* FENE spring constant, >= 0 */
    double r0_fene;       /* FENE maximum extension, > 0 */
    double eps_wca;       /* LJ energy, >= 0 */
    double sigma_wca;     /* LJ length, > 0; cut and shifted at 2^(1/6) sigma */
    uint32_t seed;        /* Philox key word 0 */
    uint32_t box_id;      /* Philox key word 1 */
    int32_t chain_len;    /* beads per chain: beads c*chain_len .. c*chain_len +
                             chain_len - 1 form chain c, bonded along the chain
                             only; LJ acts between all beads of the box (a
                             semidilute solution of N / chain_len chains,
                             Sec. III.C).  0 = one chain of n_beads.  Must
                             divide n_beads. */
} lb_box_desc;

/* Observables of one box, FP64 sums in a fixed order. */
typedef struct {
    double mass;          /* sum over nodes of rho (lattice mass units = m) */
    double j_lat[3];      /* fluid momentum, lattice units */
    double p_fluid[3];    /* fluid momentum, LJ units (j_lat / tau_lb) */
    double p_beads[3];    /* sum of m v over beads */
    double p_total[3];    /* p_fluid + p_beads + (md_dt/2) sum of the beads'
                             last coupling forces: conserved at LB-step boundaries */
    double com[3];        /* centre of mass of the box's beads (unwrapped coordinates) */
    double rg2;           /* radius of gyration squared, mean over the box's chains */
    double re2;           /* end-to-end distance squared, mean over the box's chains */
    double neg_count;     /* number of populations n_i < 0 */
    double mode_sq[19];   /* sum over nodes of (m_k - rho0 delta_k0)^2 */
    uint32_t health;      /* LB_HEALTH_* bits accumulated since init (sticky) */
    uint32_t nlist_builds;/* chain neighbour-list builds since init (diagnostic) */
    uint64_t step;        /* LB steps taken since init */
} lb_obs;

/* Device bytes the caller must provide for the boxes (Sec. II.E: a cubic
 * periodic box of L^3 sites per chain; Sec. III.C: several such boxes).
 * state_bytes: two population buffers of 19 values per site (the D3Q19
 * velocity set of Sec. II.B, stored as deviations n_i - w_i rho0, FP64 or
 * FP32 per `precision`) plus bead x, v, F and coupling force; scratch_bytes:
 * node impulses, tables, reduction partials.  hist_steps >= 0: depth of the
 * ring of bead velocities kept at the end of each LB step (0 = none).  Both
 * outputs are host size_t the caller owns.  Fails with LB_EINVAL on an invalid
 * box description (ranges listed in lb_box_desc) or a NULL output pointer;
 * nothing is written then. */
lb_status lb_query_sizes(const lb_box_desc* boxes, int32_t n_boxes, int32_t precision,
                         int32_t hist_steps, size_t* state_bytes, size_t* scratch_bytes);

/* Set up the boxes of Sec. II.E (cubic, periodic, fluid density rho0, the
 * relaxation rates and kT of Sec. II.B, FENE and LJ parameters of Sec. II.A,
 * MD step md_dt and LB step tau_lb): fluid at rest at n_i = w_i rho0
 * (deviations zero), beads at bead_x0 (host, [sum N][3] FP64, boxes in order,
 * unwrapped coordinates, read once and not kept), velocities zero, last force
 * = conservative force (the FENE + LJ force of Sec. II.A).  d_state and
 * d_scratch: caller-owned device buffers of lb_query_sizes bytes, 256-byte
 * aligned; both are cleared here.  bead_x0 may be NULL only when every box has
 * N = 0.  LB_EINVAL for an invalid box, NULL or unaligned buffers, or an
 * initial bond >= R0 (the FENE potential is undefined there); LB_EDEVICE if a
 * HIP call fails.  On failure *out is NULL and nothing needs freeing.
 * stream: hipStream_t as void*, NULL = the library creates one. */
lb_status lb_init(const lb_box_desc* boxes, int32_t n_boxes, int32_t precision, int32_t hist_steps,
                  const double* bead_x0, void* d_state, void* d_scratch, void* stream,
                  lb_handle** out);

/* The coupling of Sec. II.B (coupling paragraph) for one LB step: the
 * md_substeps MD steps (Sec. II.E, time steps) of every chain in the fluid
 * velocity frozen at the current (pre-collision) state, interpolated
 * trilinearly from the surrounding sites; the friction force -zeta (v - u)
 * and the Langevin force act on each bead, and their momentum is taken from
 * the same sites.  The node impulses accumulate on the device; the fluid is
 * not updated.  The next lb_step consumes these impulses instead of coupling
 * again.  Asynchronous on the handle's stream.  LB_ESTATE if called twice
 * without an lb_step between, LB_EDEVICE on a launch failure. */
lb_status lb_couple(lb_handle* h);

/* n_steps full LB steps, each the coupling above followed by the LB equation
 * of Sec. II.B: every site's populations are collided in mode space (stress
 * modes relaxed toward the second-order equilibrium, ghost modes relaxed,
 * each non-conserved mode given noise of the variance the
 * fluctuation-dissipation theorem fixes, the node impulse applied), then
 * moved to the neighbour along c_i (periodic).  One LB step is tau_lb =
 * md_substeps * md_dt (Sec. II.E, time steps).  n_steps >= 0.  Asynchronous on
 * the handle's stream; numeric trouble sets the health word.  LB_EINVAL for
 * n_steps < 0, LB_EDEVICE on a launch or graph failure. */
lb_status lb_step(lb_handle* h, int64_t n_steps);

/* Observables of every box into out[n_boxes] (host, caller-owned): the
 * conserved mass and momentum of the LB equation (Sec. II.B: the collision
 * conserves rho and the momentum; the coupling conserves the total), the
 * chain's R_g^2 and R_e^2 and centre of mass (Sec. III.A), mode sums and the
 * count of negative populations (Sec. II.E, choice of parameters: the step is
 * chosen so that they stay rare).  FP64 sums in a fixed order, so repeated
 * calls on one state give identical bits.  Synchronises the stream.  Returns
 * LB_ENUMERIC (and still fills out) if a health bit is set, LB_EINVAL for
 * NULL arguments, LB_EDEVICE on a HIP failure. */
lb_status lb_observables(lb_handle* h, lb_obs* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * observables of lb_observables, with the partial sums of the reduction in a
 * device array the library holds statically (LB_STATIC_SCRATCH_BYTES per
 * device, from the first lb_init on that device until the process ends)
 * instead of the handle's scratch buffer.  Allocates nothing.  Same kernels
 * and summation order as lb_observables, so the same bits.  The partials
 * take 192 bytes per 4096 nodes of each box (rounded up per box) plus 12.5
 * KB per box; LB_ENOMEM if they exceed the array (the message gives both
 * sizes), LB_EDEVICE if the array's device address could not be found at
 * init.  Every call on one device shares that device's array: calls that
 * overlap on one GPU (other threads, other handles) race.  Every partial is
 * written before it is read, so nothing carries over between calls.
 * Synchronises the handle's stream. */
#define LB_STATIC_SCRATCH_BYTES ((size_t)8 << 20)
lb_status lb_observables_static(lb_handle* h, lb_obs* out);

/* Canonical state as FP64 host data, per box in order: 19 planes of L^3 full
 * populations n_i(r, t) of the LB equation (Sec. II.B; pre-collision, plane-
 * major, node r = x + L (y + L z)), then N x 3 each of bead x, v, last total
 * force, last coupling force; preceded by one uint64 step count.
 * lb_state_host_bytes gives the size; host_buf is caller-owned.  LB_ENOMEM if
 * bytes is too small, LB_ESTATE (import) with impulses pending, LB_ENUMERIC
 * (export, buffer still filled) if a health bit is set.  Synchronises the
 * stream.
 * Both storages keep deviations n_i - w_i rho0 on the device: an import of
 * exported FP32 deviations restores them exactly; FP64 deviations come back
 * to the last bit of n_i (import then export returns the same n_i wherever
 * n_i lies within a factor 2 of w_i rho0, where the subtraction is exact).
 * lb_import_state restarts the neighbour lists and fix-up stamps. */
size_t lb_state_host_bytes(const lb_handle* h);
lb_status lb_export_state(lb_handle* h, void* host_buf, size_t bytes);
lb_status lb_import_state(lb_handle* h, const void* host_buf, size_t bytes);

/* Node impulses pending after lb_couple (the momentum the coupling of
 * Sec. II.B takes from the sites around each bead), scattered into dense host
 * arrays [3][L^3] (lattice units) per box in order; zero where no bead acted.
 * host_dense is caller-owned; LB_ENOMEM if bytes is too small.  Synchronises
 * the stream. */
lb_status lb_pending_impulse(lb_handle* h, double* host_dense, size_t bytes);

/* Bead velocities stored at the end of LB step `step` (0-based), [sum N][3]
 * FP64 host, caller-owned: the samples of the velocity autocorrelation that
 * Sec. III.B's dynamics are built from.  LB_ESTATE without a ring
 * (hist_steps = 0 at init), LB_EINVAL if that step is no longer in the ring,
 * LB_ENOMEM if bytes is too small.  Synchronises the stream. */
lb_status lb_velocity_history(lb_handle* h, int64_t step, double* host_out, size_t bytes);

/* Bead positions at the current LB-step boundary, unwrapped (a chain's
 * coordinates are continuous across the periodic boundary, Sec. II.A),
 * [sum N][3] FP64 host, boxes in order.  Waits for the handle's stream.
 * LB_ESTATE between lb_couple and lb_step (the positions are mid-step). */
lb_status lb_bead_positions(lb_handle* h, double* host_out, size_t bytes);

/* Launch structure of lb_step (the arithmetic is that of lb_step, Sec. II.B,
 * in every form): batched = 1 advances every box with one launch per kernel
 * (the default); batched = 0 launches per box (the plain form).  In batched
 * steps the 64-node segments around chains above 256 beads in boxes they do
 * not cover densely are collided beside the other nodes once the chain's
 * impulses are in; batched = 2 re-collides the chain's nodes after the
 * collide instead.  Batched steps launched directly (graph_steps = 0) of
 * boxes with chains of at most 256 beads only, no dense box and at most 2^20
 * nodes in all run each step's coupling and the re-collision of its nodes
 * on one queue, the collide beside them on the other (batched = 2, and graph
 * replays, keep the re-collision behind the collide on the handle's
 * stream).  All forms compute the same bits.
 * graph_steps > 0 records that many LB steps (rounded up to even) in a HIP
 * graph and replays it; 0 launches kernels directly.  The graphs of both
 * buffer parities are recorded and instantiated here, before returning
 * (synchronous), so that lb_step only replays them.  Exception: batched FP32
 * steps whose chains all exceed 256 beads (and cover no box densely) are
 * always launched directly: each collide there carries the step's node
 * tables and a resident chain kernel waits for them, an order that graph
 * replay does not keep (a stream under capture takes a graph-safe form).
 * Such a run also needs the GPU to run kernels of its two streams at once;
 * where a tool runs one kernel at a time (hardware counter collection), the
 * wait gives up and LB_HEALTH_SYNC is set.  batched = 3 is batched = 1
 * without that layout: the node tables get a kernel of their own, and
 * graph_steps applies.
 * LB_EINVAL for batched outside 0..3 or graph_steps < 0, LB_ESTATE with
 * impulses pending, LB_EDEVICE if capture or instantiation fails. */
lb_status lb_set_launch(lb_handle* h, int32_t batched, int32_t graph_steps);

/* ---- adjoint window (gradient of a loss of the bead velocities) ----------
 * The loss is any function J of the bead velocities recorded at the end of
 * each LB step of a window of T steps.  lb_window_backward returns, per box,
 * dJ/d(omega_shear, omega_bulk, zeta), the rates that set the fluid's shear
 * and bulk viscosity and the bead friction (Sec. II.B: relaxation of the
 * stress modes, coupling friction).  It reverses collide+stream and the
 * chain's coupling step by step by hand-written adjoint kernels, replaying
 * the noise from Philox, and rebuilds forward states from checkpoints taken
 * every k steps.  Chains of at most 256 beads.  The workspace d_ws is device
 * memory owned by the caller, lb_window_bytes(h, T, k) bytes, 256-aligned,
 * kept unchanged between the forward and backward calls.  It holds the
 * checkpoints and two tapes of k steps each, so that the backward replays one
 * segment on the handle's stream while it reverses the one after it on a
 * second stream of its own. */
size_t lb_window_bytes(const lb_handle* h, int32_t T, int32_t k);
/* Run T steps (the lb_step of Sec. II.B) from the current state,
 * checkpointing every k steps into d_ws; bead velocities after each step go to
 * vhist_host [T][sum N][3] (host, caller-owned, may be NULL).  Synchronous.
 * LB_EINVAL for T or k <= 0 or a chain above 256 beads, LB_ENOMEM for a short
 * workspace, LB_ESTATE with impulses pending. */
lb_status lb_window_forward(lb_handle* h, void* d_ws, size_t bytes, int32_t T, int32_t k, double* vhist_host);
/* Reverse sweep of the recorded window: dj_host [T][sum N][3] = dJ/dv (host,
 * read), grad_host [n_boxes][3] = dJ/d(omega_shear, omega_bulk, zeta) (host,
 * written).  The adjoint of each step reverses the LB equation and the
 * coupling of Sec. II.B in FP64.  Leaves the state at the end of the window.
 * Synchronous.  LB_ESTATE without a recorded forward window, LB_ENOMEM for a
 * short workspace. */
lb_status lb_window_backward(lb_handle* h, void* d_ws, size_t bytes, const double* dj_host, double* grad_host);
/* Restore the state at the start of the recorded window (from the first
 * checkpoint in d_ws).  LB_ESTATE without a recorded window. */
lb_status lb_window_rewind(lb_handle* h, void* d_ws, size_t bytes);
/* Change a box's shear and bulk relaxation rates (the stress-mode rates of
 * the collision, Sec. II.B) and bead friction zeta_bare (Sec. II.B, coupling
 * paragraph); the ranges are those of lb_box_desc, else LB_EINVAL.
 * Synchronises the stream; takes effect at the next step. */
lb_status lb_set_rates(lb_handle* h, int32_t box, double omega_shear, double omega_bulk, double zeta);

/* Benchmark aid: enqueue n launches of the fused collide+stream kernel (the
 * LB equation of Sec. II.B at every site) of every box from the current state
 * into the other buffer, with no impulses and without advancing the state
 * (the other buffer is overwritten by the next step anyway).  Lets a caller
 * time the dominant kernel with events on the handle's stream.  LB_EINVAL for
 * n < 0. */
lb_status lb_collide_only(lb_handle* h, int32_t n);

/* ---- launch-shape autotuning of the collide+stream kernel ---------------
 * LB_N_COLLIDE_VARIANTS launch shapes compute identical values (same per-node
 * arithmetic, bit for bit); they differ in the cap on resident waves per SIMD
 * (4..8), in the nodes per workgroup and in the grid: one workgroup per
 * 256-node tile (variants 0..4, at most 4..8 waves per SIMD), a grid of
 * n_CU x waves workgroups that strides over the tiles (5..9), one workgroup
 * per 512 nodes (10: at most 4 waves per SIMD; 11: at most 6) or per 1024
 * nodes (12).
 * lb_autotune times every variant on the handle's own state (two sweeps; in
 * each, reps launches per variant after two untimed ones, HIP events on the
 * handle's stream, no state change), selects the fastest, drops recorded
 * graphs (recording them again for the chosen shape), and writes each
 * variant's faster sweep average in microseconds per launch to
 * times_us[LB_N_COLLIDE_VARIANTS] (may be NULL) and the choice to *chosen (may
 * be NULL).  lb_set_collide_variant forces one (LB_EINVAL out of range).
 * The arithmetic is the LB equation of Sec. II.B in every shape. */
#define LB_N_COLLIDE_VARIANTS 13
lb_status lb_autotune(lb_handle* h, int32_t reps, float* times_us, int32_t* chosen);
lb_status lb_set_collide_variant(lb_handle* h, int32_t variant);

/* Plumbing, no paper passage: the stream the handle enqueues on (hipStream_t
 * as void*); lb_free waits for the handle's work and releases its host
 * metadata, graphs and own streams (never caller memory; NULL is a no-op);
 * lb_last_error gives the message of the last failing call on h (NULL: of
 * the calling thread's last lb_query_sizes / lb_init failure). */
void* lb_stream(const lb_handle* h);

void lb_free(lb_handle* h);
const char* lb_last_error(const lb_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* LBMD_H */
