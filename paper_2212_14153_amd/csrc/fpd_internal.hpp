// fpd_internal.hpp -- structures shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fpdlbm.h"

namespace fpd {

constexpr int kMaxBeads = FPD_MAX_BEADS;
constexpr int kBeadThreads = 256;   // finish kernel (one thread per bead)
// The per-bead FP64 sums of the bead kernels run over kBeadLanes virtual lanes in a fixed
// order (each lane's nodes in increasing order, a wave tree per 64 lanes, then the waves in
// order), whatever the block size; a real thread carries kBeadLanes / blockDim of them.
// One simulation launches kBeadBlock threads per bead (few blocks: latency bound), a batch
// kBatchBeadBlock (thousands of blocks: throughput bound), and a simulation's bead
// velocities are bitwise the same alone and in a batch.
constexpr int kBeadLanes = 512;
constexpr int kBeadBlock = 512;
constexpr int kBatchBeadBlock = 256;
static_assert(kBeadLanes % kBeadBlock == 0 && kBeadLanes % kBatchBeadBlock == 0 &&
                  kBatchBeadBlock % 64 == 0 && kBeadBlock % 64 == 0,
              "bead blocks must divide the virtual lanes into whole waves");
// block of the driven-particle diagnostics (one block, a plain block reduction)
constexpr int kStatsBlock = 256;
// nodes per thread and pass of the velocity sums: one simulation (few bead blocks, latency
// bound: 4) and batches (thousands of bead blocks, where fewer registers let more blocks
// reside: 2; the FP16 sweep step 590 -> 580 us); the sums run in the same order for any
// value, so batched and single results stay bitwise equal
constexpr int kBeadVelBatch = 4;
constexpr int kBatchBeadVelBatch = 2;
// Occupancy bitmap of the fiber supports: one bit per square cell of 2^occ_shift nodes.
constexpr int kOccWords = 1024;   // up to 32768 cells per slot

// Device-resident fiber state, float64 (bead integration and reductions stay in FP64
// whatever the population storage).
struct BeadState {
    double R[kMaxBeads][2];   // positions R_i^n
    double V[kMaxBeads][2];   // V_i^n, velocity of the last step
    double F[kMaxBeads][2];   // F_i^n, Eqs. (10)-(12) (written by the owner tile)
    double C[kMaxBeads][2];   // F_i^n / A_i^n, the coefficients of Eq. (4)
    double A[kMaxBeads];      // A_i^n = sum_x phi_i^n(x)
    // Support window of phi as raw bounds (lo, hi) of node columns (unwrapped) and
    // (j0, j1) of rows, one slot per buffer parity: the bead kernel of a step fills the
    // slot the next step reads with atomic min / max, so the result does not depend on the
    // order in which beads finish.
    int win[2][4];
    // Cells any bead's support touches, one bitmap per parity like the window: the bead
    // kernel marks the slot the next step reads (atomic or), tile 0 of a step clears the
    // slot the step's bead kernel fills.  Only tiles over a marked cell gather beads.
    unsigned int occ[2][kOccWords];
    unsigned int health;                 // FPD_HEALTH_* bits, sticky (atomic or)
    unsigned int reserved;
    unsigned long long max_strain_bits;  // bits of the largest |L - l0| / l0 (atomic max)
    // excluded volume between fibers: strength (0: off) and range (set with the fiber),
    // and each bead's share of it at the step's start (ev_kernel, read by the tiles)
    double ev_k, ev_d;
    double Fev[kMaxBeads][2];
    // Partition of a split step, one slot per parity like the window: columns x0 + [0, w)
    // and rows y0 + [0, h) (modulo the lattice along periodic directions; w = 0: empty),
    // the step's support window grown by kPartMargin nodes, written by the step before.
    int part[2][4];
};

// A bead moves less than one node per step (0.3 c_s raises FPD_HEALTH_MACH long before),
// so the support window of step n grown by one node holds that of step n + 1, and one more
// node holds the ring around it that the bead kernel of step n + 1 pulls from; the third
// is slack.
constexpr int kPartMargin = 3;

// The tiles of a step: all of them (one kernel), or those outside the step's partition
// (kPartFluid: no fiber work, so the bead kernel of the step before may still be running)
// and those inside it (kPartFiber: the fiber tiles and the step's bookkeeping).
enum { kPartAll = 0, kPartFluid = 1, kPartFiber = 2 };

// Value (k, y, x) of a population buffer sits at y * stride + k * plane + x.  The nine
// direction rows of one lattice row are adjacent (plane = nx padded to 64 elements, stride
// = 9 * plane): the streams of a tile stay within a few hundred KB of each other.
// Nodes one lane of the lattice kernel updates along x: two for 2-byte storage (the
// populations move as 32-bit words), one otherwise.  The group code also takes four
// (64-bit vectors); on MI355X that was 14 % slower at 8192 x 2048 (fewer resident waves).
constexpr int nodes_per_lane(int storage) {
    return (storage == FPD_F16DEV || storage == FPD_BF16DEV) ? 2 : 1;
}

struct Lattice {
    int nx, ny, stride;       // stride: row pitch in elements
    int periodic;             // 1: no walls, y wraps like x (FPD_PERIODIC)
    long long plane;          // offset between directions k and k + 1 in elements
};

// What the kernels need to evaluate phi, eta and the force density near the fiber.
struct Fiber {
    BeadState* bs;
    int n;                    // beads (0: no fiber)
    int chain_len;            // beads per fiber: fiber c is beads c L .. c L + L - 1
    int occ_shift;            // occupancy cell side 2^occ_shift nodes
    int occ_nx, occ_ny;       // cells per row and rows of cells
    double a, xi, inv_xi;     // radius and interface thickness
    double rc, rc2;           // support radius a + cutoff * xi and its square
    double nu_f, nu_s;        // fluid and solid kinematic viscosity (rho0 = 1)
    double s_q_fixed;         // > 0 fixed heat-flux rate, else the magic per-node value
    int clamp;                // clamp sum phi <= 1
    void* rect_f;             // force density f^n on the support window, [h][w][2] of T
    int rect_wmax, rect_hmax; // reserved window
    double l0, ks_l02, kb;    // spring rest length, k_s / l0^2, k_b
    double fext[2];           // external force on every bead
};

struct StepArgs {
    int parity;               // index of the source buffer: the window slot of step n
    const void* src;          // post-collision populations of step n-1
    void* dst;                // post-collision populations of step n
    Lattice L;
    double u6;                // U / 6 (moving-wall momentum on the diagonals)
    double s_nu_f, s_q_f;     // fluid shear and heat-flux rates away from the fiber
    double s_e, s_eps;
    double gx, gy;            // uniform body force density on every node
    const double* row_phi;    // NULL or [ny]: fixed profile phi_s(y) added in Eq. (1)
    struct RecordBuf* rec;    // NULL or the fiber-ends recorder
    Fiber fib;
    int tiles_x, n_tiles;     // tiling of the fused lattice kernel
    int rows_per_block;       // block_y * rows_per_thread
    int xcd_remap;
    int part_gw, part_gh;     // grid of the kPartFiber kernel in tiles (its blocks: gw * gh)
};

// Fiber-ends recorder (device memory): at the start of every step tile 0 counts the step
// and, every `every` steps, stores the end-to-end vector R_last - R_first and the centroid
// of each fiber of the state R^n into a ring of `cap` records [step, (ex, ey, cx, cy) per
// fiber] (the step relative to the start of the recording).
struct RecordBuf {
    unsigned long long count;  // steps seen since the start
    int every, cap, fibers, pad;
    double data[1];            // [cap][1 + 4 * fibers]
};

// A work item of a batch kernel: its simulation's row in the tables and its index within
// that simulation (tile or bead); one 8-byte entry, so a block finds both in one load.
struct ItemRef {
    int sim, local;
};

// A batch step: per simulation two StepArgs (the step parities of a chunk), item tables
// and counts {simulations, tiles, beads}; all in device memory, so a captured graph stays
// valid while the tables are rewritten with the same counts (the grids are sized from the
// counts at launch).
struct BatchArgs {
    const StepArgs* args;       // [2 * n]
    const ItemRef* tile_items;  // [tiles]: simulation and tile of each lattice item
    const ItemRef* bead_items;  // [beads]: simulation and bead of each bead item
    const int* counts;          // [3]
    int gpar;                   // parity of this step within the chunk
};

// A box of nodes: columns cx0 + [0, cw) and rows cy0 + [0, ch), modulo the lattice along
// periodic directions.  A box that spans a whole period along a direction (wrap_x: cw ==
// nx; wrap_y: ch == ny in a periodic box) wraps onto itself there: neighbour lookups
// inside it are then taken modulo its size.  Otherwise its one-node border only feeds
// the gradient stencil of the nodes inside.
struct NodeBox {
    int cx0, cw, cy0, ch;
    bool wrap_x, wrap_y;
};

// Kernel launchers (fpd_kernels.hip).  Given events t0 and t1, the lattice and bead
// launches stamp them with the dispatch's own start and end (hipExtLaunchKernel); they are
// then not for stream capture.
hipError_t launch_step(int storage, const StepArgs& a, dim3 block, int rows_per_thread,
                       hipStream_t st, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
// One half of a split step (kPartFluid or kPartFiber; the fiber half's grid is
// a.part_gw * a.part_gh blocks)
hipError_t launch_step_part(int storage, const StepArgs& a, dim3 block, int rows_per_thread,
                            int part, hipStream_t st, hipEvent_t t0 = nullptr,
                            hipEvent_t t1 = nullptr);
hipError_t launch_bead(int storage, const StepArgs& a, int do_velocity, int win_out,
                       hipStream_t st, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_forces(const StepArgs& a, hipStream_t st);
// excluded-volume forces of the step's start into BeadState::Fev (before the lattice step;
// needed only when BeadState::ev_k > 0)
hipError_t launch_ev(const StepArgs& a, hipStream_t st);
// fiber-ends record of the step about to run (nothing unless a recording runs)
hipError_t launch_record(const StepArgs& a, hipStream_t st);
// any_periodic: some simulation of the batch has no walls (the kernel then reads the
// boundary of each simulation from its arguments)
hipError_t launch_batch_step(int storage, const BatchArgs& b, dim3 block, int rows_per_thread,
                             const int counts[3], bool any_periodic, hipStream_t st);
hipError_t health_gather(BeadState* const* states, unsigned* out, int n, hipStream_t st);
hipError_t launch_unstream(int storage, const Lattice& L, double u_wall, const double* f64,
                           void* dst, hipStream_t st);
hipError_t launch_stream_out(int storage, const Lattice& L, double u_wall, const void* src,
                             double* f64, hipStream_t st);
hipError_t launch_init_eq(const Lattice& L, double u_wall, int init_flow, double* f64,
                          hipStream_t st);
// allocation-free set-up (fpd_run_static): the initial state written straight into a
// population buffer (the values init_eq + unstream give), an 8-byte zero fill (bytes a
// multiple of 8), a fresh fiber from device positions R [n][2] into a zeroed bead state,
// and positions (device [n][2]) plus health bits (device, may be NULL) out of a bead state
hipError_t launch_init_state(int storage, const Lattice& L, double u_wall, int init_flow,
                             void* dst, hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_fiber_setup(BeadState* bs, const double* R, int n, double ev_k, double ev_d,
                              hipStream_t st);
hipError_t launch_beads_out(const BeadState* bs, int n, double* R, unsigned* health,
                            hipStream_t st);
hipError_t launch_fields(int storage, const StepArgs& a, double* rho, double* ux,
                         double* uy, double* eta, hipStream_t st);
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t st);
// fields[4 * cw * ch] (device scratch), out[8] (device)
hipError_t launch_particle_stats(int storage, const StepArgs& a, int bead, const NodeBox& B,
                                 double* fields, double* out, hipStream_t st);

}  // namespace fpd
