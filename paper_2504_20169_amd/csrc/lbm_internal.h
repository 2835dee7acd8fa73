// Internal structures shared by the kernels (lbm_kernels.hip) and the runtime (lbm_capi.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_lattice.h"

namespace lbm {

enum Side { XMIN = 0, XMAX = 1, YMIN = 2, YMAX = 3 };
enum Bc { BC_PERIODIC = 0, BC_ZG = 1, BC_NRBC = 2, BC_NRBC_A = 3 };

// Sides with the characteristic fill (the perfectly non-reflecting LODI boundary, or CBC (A)).
inline __host__ __device__ bool is_char_bc(int b) { return b == BC_NRBC || b == BC_NRBC_A; }
enum Storage { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2 };

// Device descriptor of one run.  Lives in device memory (one per run); kernels receive an
// array of pointers to descriptors, so a single run and a batch share every kernel.
//
// Grid: Nx x Ny nodes; population i of node (x, y) is f[par][i * plane + y * pitch + x].  With
// the row layout (default) the q population rows of one grid row are adjacent (plane = padded
// row, pitch = q padded rows), which keeps the pulls of a tile inside a few MiB of address
// space; with the plane layout `plane` is a whole padded plane and `pitch` a padded row.
// Arrays of per-pair and per-shell constants are sized for the largest stencil (D2Q37).
// Frame: the nodes outside the fast interior rectangle [fx0,fx1) x [fy0,fy1), i.e. a frame of
// depth gxm/gxp/gym/gyp on the four sides.  The ring is the outer part of the frame with depth 3
// on characteristic (NRBC) sides only: the boundary nodes that need the FP64 characteristic
// fill, handled by the first blocks of the boundary launches.  Strips of a frame-shaped region
// are numbered bottom strip, top strip, left strip, right strip (row-major inside each strip).
// Frame index t, which Q and the moment strips U use: the ring nodes first, t = their ring index
// in [0, ring_n); then, from ann0 (ring_n rounded up to 64) on, the other frame nodes, numbered
// as the strips of the annulus between the ring's inner rectangle and the fast rectangle (depths
// axm/axp/aym/ayp); the ring_n..ann0 gap is unused.  A frame thread touches its own Q/U entries
// with unit stride, and the ring blocks and the frame blocks share no cache line of Q or U.
// Without a ring the numbering is the frame's own strip numbering.
struct alignas(256) RunDev {
    int Nx, Ny, pitch, storage;
    long long plane;          // element stride between populations of one node
    long long fsize;          // elements of one population buffer
    long long qplane;         // elements per component plane of Q and U
    int gxm, gxp, gym, gyp;   // frame depths
    int Wxm, Wxp, Wym, Wyp;   // PML width per side (0 if none)
    int W, qd, open_x, open_y;
    int bc[4];
    int fx0, fx1, fy0, fy1;   // fast rectangle
    int frame_n, has_q, ring_n, pml_terms;   // pml_terms: PML moments in the NRBC target
    int rxm, rxp, rym, ryp;   // characteristic-boundary ring depths (3 on NRBC sides, else 0)
    int axm, axp, aym, ayp;   // depths of the frame's annulus off the ring
    int ann0, ann_n;          // first frame index and count of the frame nodes off the ring
    int tiles_x[3], tiles_y[3];   // bulk tiles for tile widths 64, 128, 256
    // state
    void *f[2];
    void *Q;                  // [q][qplane] in the compute type
    double *U[2];             // [4][qplane]: rho, ux, uy, T (absolute values)
    void *G;                  // [q][rplane] compute type: post-boundary populations of the ring
    double *P;                // [4][rplane]: characteristic targets formed by k_target (if tgt_pre)
    long long rplane;
    int par, tgt_pre;         // tgt_pre: NRBC targets formed by k_target (PML moments or CBC (A))
    long long step, limit;    // a run is active while step < limit
    // constants (double and float copies)
    double omega, rho0, u0x, u0y, T0, th0, b0, r0x, r0y, sigma_max, inv_W2, scale, inv_scale;
    double H0rest, H0e[NPAIR_MAX], H0o[NPAIR_MAX], E2_0[NSHELL_MAX], O1_0[NSHELL_MAX];
    float omega_f, rho0_f, u0x_f, u0y_f, th0_f, b0_f, r0x_f, r0y_f, T0_f, scale_f, inv_scale_f;
    float H0rest_f, H0e_f[NPAIR_MAX], H0o_f[NPAIR_MAX], E2_0_f[NSHELL_MAX], O1_0_f[NSHELL_MAX];
#ifdef LBM_BOUNDS
    unsigned oob;             // bounds-checked build: nonzero once a kernel met an index out of range
#endif
};

// Launch decomposition of a set of runs: prefix[k] = first block of run k, prefix[n] = total.
// Classes: the interior tiles; the frame launch (ring blocks, then frame blocks); the phase-A
// launch (ring blocks, then frame blocks if the run has a PML); the characteristic targets of
// runs that select the PML moments (ring blocks).
enum Cls { CLS_BULK = 0, CLS_FRAME = 1, CLS_A = 2, CLS_TGT = 3, NCLS = 4 };
struct KernelSet;
struct LaunchSet {
    const KernelSet *ks;      // kernels of the runs' velocity stencil (one stencil per set)
    RunDev *const *runs;      // device array of descriptor pointers
    const int *prefix[NCLS];  // device prefix arrays per class
    int blocks[NCLS];         // total blocks per class
    int nruns;
    int poison = 0;           // debug canary: NaN-fill each step's destination buffers first
    int split = -1;           // fused grid: phase-A blocks after split/8 of the tiles; -1 default
};

constexpr int FRAME_BLOCK = 256;
// Ring nodes per block of the boundary launches: one active wave per 256-thread block, so the
// ring's few, poorly coalesced waves (a 3-wide strip puts ~21 grid rows in one wave) land on
// different compute units instead of sharing one unit's memory pipeline four at a time.
constexpr int RING_BLOCK = 64;

// Blocks of a run in the boundary launches: ring blocks, then frame blocks, each count rounded up
// to a multiple of 8.  Blocks are dealt round-robin to the 8 XCDs, so every run's frame blocks
// then start on the first XCD and can be remapped XCD by XCD (neighbouring strip rows, which
// share pulled rows and Q planes, on one XCD and its L2); the padding blocks exit at once.
__host__ __device__ inline int ring_block_count(int ring_n) {
    return ((ring_n + RING_BLOCK - 1) / RING_BLOCK + 7) & ~7;
}
__host__ __device__ inline int frame_block_count(int frame_n) {
    return ((frame_n + FRAME_BLOCK - 1) / FRAME_BLOCK + 7) & ~7;
}

// Kernel launchers of one velocity stencil (lbm_kernels.hip, compiled once per stencil).  All
// enqueue on `s` and return the HIP status of the launch.
// phase_a: characteristic fill of the ring and PML auxiliary update; frame: phase B (collision)
// of every frame node, ring included; target: characteristic targets with the PML moments.
struct KernelSet {
    int q;
    // step kernels of sub-step ks of a batch (parity par + ks; active while step + ks < limit)
    hipError_t (*phase_a)(const LaunchSet &L, int storage, int ks, hipStream_t s);
    // frame, phase_a_bulk and bulk take optional events a and b (both or neither), attached to
    // the dispatch: they take the kernel's own start and end time
    hipError_t (*frame)(const LaunchSet &L, int storage, int ks, hipStream_t s, hipEvent_t a,
                        hipEvent_t b);
    hipError_t (*target)(const LaunchSet &L, int storage, int ks, hipStream_t s);
    // phase A and the bulk tiles in one launch
    hipError_t (*phase_a_bulk)(const LaunchSet &L, int storage, int tx, int ks, hipStream_t s,
                               hipEvent_t a, hipEvent_t b);
    hipError_t (*bulk)(const LaunchSet &L, int storage, int tx, int ks, hipStream_t s,
                       hipEvent_t a, hipEvent_t b);
    // end of a batch of n sub-steps: step counters and parities advance
    hipError_t (*advance)(const LaunchSet &L, int n, hipStream_t s);
    hipError_t (*set_limit)(RunDev *run, long long limit, hipStream_t s);
    hipError_t (*set_limits)(RunDev *const *runs, const long long *limits, int n, hipStream_t s);
    hipError_t (*init)(RunDev *run, int storage, int Nx, int Ny, const double *rho,
                       const double *ux, const double *uy, const double *T, float *absmax,
                       hipStream_t s);
    hipError_t (*moments)(RunDev *run, int storage, int Nx, int Ny, double *rho, double *ux,
                          double *uy, double *T, hipStream_t s);
    hipError_t (*export_f)(RunDev *run, int storage, int Nx, int Ny, const double *fbar,
                           double *out, hipStream_t s);
    // Q of every frame node into a full grid (nt: the frame index extent, ann0 + ann_n)
    hipError_t (*export_q)(RunDev *run, int storage, int nt, double *out, hipStream_t s);
    hipError_t (*check)(RunDev *run, int storage, int Nx, int Ny, int *flag, hipStream_t s);
    hipError_t (*err_rows)(const double *rho, const double *ux, const double *T, int Nx,
                           int x0, int y0, int lx, int ly, const double *rr, const double *ru,
                           const double *rt, double *partials, hipStream_t s);
    // the sums of err_rows over the moments of the run's current state, formed in the kernel
    hipError_t (*err_rows_state)(RunDev *run, int storage, int x0, int y0, int lx, int ly,
                                 const double *rr, const double *ru, const double *rt,
                                 double *partials, hipStream_t s);
    hipError_t (*err_final)(const double *partials, int nrows, double *out, hipStream_t s);
    // debug canary of sub-step ks: NaN into the buffers the step writes in full (every active run)
    hipError_t (*poison)(const LaunchSet &L, int storage, int ks, hipStream_t s);
};

namespace k37 { extern const KernelSet kernels; }
namespace k17 { extern const KernelSet kernels; }
namespace k9 { extern const KernelSet kernels; }

}  // namespace lbm
