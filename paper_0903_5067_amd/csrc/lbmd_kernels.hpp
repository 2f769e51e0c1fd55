// Launch interface between the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lbmd_device.hpp"

namespace lbd {

// Device pointers and sizes every launcher needs; filled by the runtime.
struct LaunchCtx {
    hipStream_t stream;
    int n_cu;                      // compute units of the device
    int collide_variant;           // launch shape of the collide kernel (0..N_COLLIDE_VARIANTS-1)
    const BoxDev* boxes;
    const BoxDev* boxes_host;      // host copy of the box table
    int n_boxes;
    const void* ccs;               // CollideConst<R>[n_boxes]
    const uint32_t* tile_box;      // box index of every collide tile
    Ctrl* ctrl;
    unsigned long long* imp;       // dense node impulses, 3 per global node, fixed point 2^-52
    uint32_t* claim;               // per global node: step stamp of the last fix-up
    uint32_t* touched;             // per bead: touch_cap slots of local node ids
    int32_t* touched_cnt;          // per bead
    int touch_cap;                 // touched slots per bead
    uint32_t* nl_rebuilds;         // per box: neighbour-list builds (diagnostic)
    const int32_t* bead_box;       // box index of every bead
    double *x, *v, *f, *fc;        // beads [total][3]
    int32_t* nl_cnt; uint16_t* nl_idx; double* nl_x0; int nl_cap;
    double* vhist; int hist_len; uint64_t total_beads;
    double* tape;                  // substep tape while replaying an adjoint window segment (else null)
    double* tape_x0;               // with tape: the step's starting bead x; v and f follow at tape_vo, tape_fo
    uint64_t tape_vo, tape_fo;     // (in doubles), the state's own layout
    int keep_imp;                  // 1: the fix-up leaves the node impulses in place (adjoint replay records them)
    // chains above BIG_CHAIN beads
    void* near_u;                  // [total beads][27][3] node velocities around each bead (storage precision)
    int4* near_c;                  // [total beads] nearest node the table is centred on
    double* sub_rec;               // [most substeps][total beads][8] per-substep records
    void* field;                   // dense boxes: node velocities (MD units, storage precision) [nodes][3]
    uint32_t dense_max_tiles;      // collide tiles of the largest dense box (0: none)
    int big_sparse;                // boxes on the 1024-thread path that are not dense (k_spread's boxes)
    uint32_t* bin_start;           // dense boxes: per base node, first binned stencil run [L^3 + 1]
    unsigned long long* runimp;    // dense boxes: per stencil run, the fixed-point impulse to its 8 corners x 3
    uint32_t* slot_of;             // dense boxes: per bead and run, the run's slot [N x substeps]
    // deferred segments: in a batched step the 64-node segments (wavefronts
    // of the collide tiles) that hold a node of any table of a sparse box's
    // large chain are left out of the plain collide and collided with their
    // impulses beside it, once the coupling is done; impulses that land
    // outside them are listed for a fix-up
    int defer_on;                  // this launch defers (the pointers below are always set)
    uint32_t* defer;               // per segment and step parity: stamp of the last step that deferred it
    uint32_t* dclaim;              // per segment: stamp of the last step that listed it
    uint32_t* defer_list;          // the deferred segments, Ctrl::defer_cnt of them
    uint32_t defer_cap;
    uint32_t* ovf;                 // (bead, local node) pairs, Ctrl::ovf_cnt of them
    uint32_t ovf_cap;
    uint32_t* ovm;                 // per global node: stamp of the last step that listed it in ovf
};

template <typename R>
hipError_t launch_collide(const LaunchCtx& c, const void* A, void* B, int fixed_box, uint32_t tile0,
                          uint32_t n_tiles, uint32_t s_off);
template <typename R>
hipError_t launch_fixup(const LaunchCtx& c, const void* A, void* B, uint64_t bead0, uint64_t n_beads,
                        uint32_t s_off);
// the deferred tiles' collide (after the coupling, beside the plain
// collide) and the end-of-step pass: fix-up of the listed impulses outside
// them, then the deferral cleared
template <typename R>
hipError_t launch_collide_deferred(const LaunchCtx& c, const void* A, void* B, uint32_t s_off);
// advance: added to the device step counter once the fix-up is done (0: none)
template <typename R>
hipError_t launch_overflow(const LaunchCtx& c, const void* A, void* B, uint32_t s_off, uint32_t advance = 0);
template <typename R>
hipError_t launch_collide_forced(const LaunchCtx& c, const void* A, void* B, int fixed_box, uint32_t tile0,
                                 uint32_t n_tiles, uint32_t s_off);
template <typename R>
hipError_t launch_couple(const LaunchCtx& c, const void* A, const int32_t* list, int n_list, int block,
                         uint32_t s_off);
// chains of BIG_CHAIN+1..1024 beads (at most max_n): one 1024-thread workgroup
// per box in `list`, with its node-table and impulse-spreading launches.
// after_table (may be null) is recorded on c.stream between the node-table
// kernel and the chain kernel.  Aprev (batched steps that defer tiles, sparse
// boxes only): the previous step's input buffer; the node-table kernel then
// fixes up the previous step's impulses outside its deferred tiles and the
// chain kernel clears them and resets the list counts (instead of the
// end-of-step kernel of launch_overflow).
// single_box: the box `list` holds when n_list == 1 (its descriptor is then
// passed to the node-table kernel by value), or -1.
// wait_head > 0: no node-table kernel; the step's collide carries the node
// tables (launch_collide_headed) and the chain kernel waits for its wait_head
// node-table workgroups, then clears the previous step's impulses outside its
// deferred tiles.  zero_head: the node-table kernel starts a run of such
// steps (zeroes the workgroup counts).  stamp_next: the chain kernel stamps
// the next step's deferred tiles from its end positions.
template <typename R>
hipError_t launch_couple_big(const LaunchCtx& c, const void* A, const int32_t* list, int n_list, int max_n,
                             uint32_t s_off, hipEvent_t after_table, const void* Aprev = nullptr,
                             int single_box = -1, uint32_t wait_head = 0, int zero_head = 0, int stamp_next = 0);
// step s_off's plain collide over tiles 0..n_tiles-1 with the node-table work
// of the big chains in `list` in its first workgroups (their count is
// head_blocks(n_list, max_n)); Aprev: the previous step's input buffer
template <typename R>
hipError_t launch_collide_headed(const LaunchCtx& c, const void* A, void* B, uint32_t n_tiles, uint32_t s_off,
                                 const int32_t* list, int n_list, int max_n, const void* Aprev, int single_box);
constexpr int BIG_CHAIN = 256;   // chains above this many beads take the one-workgroup-per-chain kernel
constexpr int NEAR_ITEMS = 27;   // table nodes per bead
inline uint32_t head_blocks(int n_list, int max_n)
{
    return (uint32_t)n_list * (uint32_t)((max_n * NEAR_ITEMS + 255) / 256);
}
hipError_t launch_advance(const LaunchCtx& c, uint32_t n);
hipError_t launch_init_forces(const LaunchCtx& c, const int32_t* list, int n_list, int block);
// observables of the state A: per-block records in part [sum of stat_recs_of(n_tiles)][NSTAT_REC]
// (box b's from BoxDev::stat_off), per-chunk sums in mid [n_boxes][STAT_CHUNKS][NSTAT_REC], per-box
// sums in out [n_boxes][NSTAT_REC]; max_recs: the most records of any box
template <typename R>
hipError_t launch_stats(const LaunchCtx& c, const void* A, uint32_t max_recs, double* part, double* mid,
                        double* out);
hipError_t launch_chain_obs(const LaunchCtx& c, double* out);

// device pointers of one reverse step of the adjoint window
struct AdjArgsHost {
    const double *x0, *v0, *f0, *tape, *dj;
    double *lx, *lv, *lf, *lam_n;
    const double* lam_dp;
    double* gz;
    uint64_t nodes;
};
template <typename R>
hipError_t launch_adj_collide(const LaunchCtx& c, const void* ccd, const void* P, const unsigned long long* imp,
                              const double* lam_next, double* lam_cur, double* lam_dp, double* gpart,
                              uint64_t nodes, uint32_t total_tiles, uint32_t step);
template <typename R>
hipError_t launch_adj_couple(const LaunchCtx& c, const int32_t* list, int n_list, int block, const void* P,
                             const AdjArgsHost& a, uint32_t step);

constexpr int N_COLLIDE_VARIANTS = 13;
constexpr int DEFAULT_COLLIDE_VARIANT = 3;   // one block per tile, at most 7 waves per SIMD
constexpr int NSTAT_REC = 24;
constexpr int STAT_TPB = 16;      // collide tiles per block of the observables pass (16 nodes per thread)
constexpr int STAT_CHUNKS = 64;   // per box, the block records are summed in this many fixed ranges first
__host__ __device__ inline uint32_t stat_recs_of(uint32_t n_tiles) { return (n_tiles + STAT_TPB - 1) / STAT_TPB; }
constexpr int NCHAIN_REC = 11;
constexpr int NL_SLOTS = 32;
constexpr int TAPE_REC = 40;     // doubles per bead and substep in the adjoint tape

}  // namespace lbd
