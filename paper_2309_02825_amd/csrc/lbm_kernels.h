// Host-side launchers of the HIP kernels (defined in lbm_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_lattice.h"

namespace lbm {

// State layout ("chunked structure of arrays"): node indices are grouped in
// chunks of CHUNK consecutive nodes; inside a chunk the q populations follow
// one another as runs of CHUNK doubles.  Population i of node k lives at
//     ((k / CHUNK) * q + i) * CHUNK + k % CHUNK.
// With 4096-node chunks (32 KiB runs) the q read and q write streams of a
// step stay inside a few contiguous regions of HBM, which sustains a higher
// bandwidth on MI355X than q planes far apart.
constexpr int LOG2_CHUNK = 12;
constexpr int64_t CHUNK = int64_t(1) << LOG2_CHUNK;

template <int Q>
__host__ __device__ __forceinline__ int64_t slot(int i, int64_t k) {
    return (((k >> LOG2_CHUNK) * Q + i) << LOG2_CHUNK) + (k & (CHUNK - 1));
}

inline int64_t chunks_of(int64_t V) { return (V + CHUNK - 1) >> LOG2_CHUNK; }

// Launch geometry of the per-node kernels: one node per thread, 256 threads
// per block laid along x (a block covers 256 consecutive nodes of one row).
constexpr int BLOCK_X = 256;
constexpr int BLOCK_Y = 1;
constexpr int BLOCK_1D = 256;

struct Geo {
    int nx, ny, nz, nw; // nodes per axis (1 for unused axes)
    int64_t V;          // nx * ny * nz * nw
};

// Launch shape of the per-node kernels for one grid.
struct Launch {
    dim3 grid, block;
    int64_t nblocks;
};
Launch launch_shape(int d, const Geo& g);

// rin: src was written by a collision, so each twin population (twin<D>,
// lbm_lattice.h) is read from the plane of the one it equals; wout: twins
// are not stored, and dst may then only be read with rin.  Neither changes
// the result.  The defaults read and write every population.
hipError_t launch_step(int d, const Geo& g, const Rates& r, const double* src, double* dst,
                       hipStream_t st, bool rin = false, bool wout = false);
// nsteps (2, 4 or 8) D2Q9 steps in one pass over HBM (temporal blocking);
// bitwise equal to nsteps launch_step calls.  A block of MS_THREADS threads
// (one wave) produces a strip of strip_width(nsteps) columns.
constexpr int MS_THREADS = 64;
constexpr int MAX_STEPS_PER_PASS = 8;
__host__ __device__ constexpr int strip_width(int nsteps) { return MS_THREADS - 2 * nsteps; }
hipError_t launch_steps(int nsteps, const Geo& g, const Rates& r, const double* src, double* dst,
                        hipStream_t st, bool rin = false, bool wout = false);
// The same passes keeping every intermediate state: step j of the pass
// (1..nsteps) goes to out + (j - 1) stride; the buffers must not overlap src.
hipError_t launch_steps_all(int nsteps, const Geo& g, const Rates& r, const double* src,
                            double* out, int64_t stride, hipStream_t st, bool rin = false,
                            bool wout = false);
// nsteps (2) D3Q19 steps in one pass; a block of MS3_TX x MS3_TY threads
// produces a tile of tile_width3 x tile_height3 columns and marches along z.
constexpr int MS3_TX = 64, MS3_TY = 8;
constexpr int MAX_STEPS_PER_PASS_3D = 2;
__host__ __device__ constexpr int tile_width3(int nsteps) { return MS3_TX - 2 * nsteps; }
__host__ __device__ constexpr int tile_height3(int nsteps) { return MS3_TY - 2 * nsteps; }
hipError_t launch_steps3(int nsteps, const Geo& g, const Rates& r, const double* src, double* dst,
                         hipStream_t st, bool rin = false, bool wout = false);
// 1-D grids up to this many nodes run all their steps in one launch with the
// state in LDS (3 populations x 8 B x 2048 = 48 KiB).
constexpr int RESIDENT_MAX_1D = 2048;
// walls != NULL: bounded interval (see launch_step_wall1); wall_now holds the
// boundary theta of the current time and receives the last pair of walls.
hipError_t launch_step_resident1(const Geo& g, const Rates& r, const double* src, double* dst,
                                int64_t nsteps, const double* walls, double* wall_now,
                                hipStream_t st);
// 1-D interval whose end nodes carry a given theta (2 doubles at wall: left,
// right, of the time the step starts from); n >= 2.
hipError_t launch_step_wall1(const Geo& g, const Rates& r, const double* src, double* dst,
                             const double* wall, hipStream_t st);
hipError_t launch_macro_wall1(const Geo& g, const Rates& r, const double* state, double* theta,
                              double* u, double* grad, const double* wall, hipStream_t st);
hipError_t launch_get_state_wall1(const Geo& g, const double* state, double* dense,
                                  const double* wall, hipStream_t st);
hipError_t launch_wall_from_dense1(const Geo& g, const double* dense, double* wall,
                                   hipStream_t st);
hipError_t launch_init(int d, const Geo& g, const Rates& r, const double* theta0,
                       const double* grad, double* dst, hipStream_t st);
// theta (V), u (d x V) and grad theta (d x V) at the state; any may be NULL.
hipError_t launch_macro(int d, const Geo& g, const Rates& r, const double* state, double* theta,
                        double* u, double* grad, hipStream_t st);
hipError_t launch_get_state(int d, const Geo& g, const double* state, double* dense,
                            hipStream_t st);
hipError_t launch_set_state(int d, const Geo& g, const double* dense, double* state,
                            hipStream_t st);
hipError_t launch_layout_from_dense(int d, const Geo& g, const double* dense, double* buf,
                                   hipStream_t st);
hipError_t launch_layout_to_dense(int d, const Geo& g, const double* buf, double* dense,
                                 hipStream_t st);
// Burgers front end (inverse Cole-Hopf).  work holds potential_workspace
// doubles.
int64_t potential_workspace(int d, const Geo& g);
hipError_t launch_theta_from_velocity(int d, const Geo& g, double dx, double nu, const double* u0,
                                      double* work, double* theta, double* grad,
                                      hipStream_t st);
hipError_t launch_check_theta(const double* theta, int64_t n, int* flag, hipStream_t st);
// Sets *flag (atomic OR) if theta = sum_i f_i is not finite and positive at some node.
hipError_t launch_check_state(int d, const Geo& g, const double* state, int* flag,
                              hipStream_t st);

// Adjoint kernels write one partial sum of the eps-gradient per block into
// `partials`; launch_finalize then adds their sum (fixed order) to *g_eps.
hipError_t launch_macro_adjoint(int d, const Geo& g, const Rates& r, const double* state,
                                const double* g_theta, const double* g_u, double* lambda,
                                double* partials, hipStream_t st);
// partials: a table of ntab >= launch_shape(d, g).nblocks entries, all written.
// rin: state was written by a collision (twins read from their partners'
// planes, as for launch_step).
hipError_t launch_adjoint_step(int d, const Geo& g, const Rates& r, const double* state,
                               const double* lam_in, double* lam_out, double* partials,
                               int64_t ntab, hipStream_t st, bool rin = false);
hipError_t launch_init_adjoint(int d, const Geo& g, const Rates& r, const double* theta0,
                               const double* grad, const double* lambda0, double* g_theta0,
                               double* g_grad, double* partials, hipStream_t st);
// With g_nu != NULL it then also writes *g_nu = nu_scale * *g_eps.
hipError_t launch_finalize(const double* partials, int64_t n, double* g_eps, hipStream_t st,
                           double* g_nu = nullptr, double nu_scale = 0.0);
// nsteps (2 or 4) D2Q9 adjoint steps in one pass: lam_out = lambda^{N-nsteps}
// from lam_in = lambda^N, with f^{N-j} at ftop - (j-1) stride; writes a table of
// exactly ntab eps partials (ntab >= adjoint_steps_table(g)).  lam_out is
// bitwise nsteps launch_adjoint_step calls.
constexpr int MAX_ADJOINT_STEPS_PER_PASS = 4;
int64_t adjoint_steps_table(const Geo& g);
hipError_t launch_adjoint_steps(int nsteps, const Geo& g, const Rates& r, const double* lam_in,
                                double* lam_out, const double* ftop, int64_t stride,
                                double* partials, int64_t ntab, hipStream_t st, bool rin = false);
// m tables of n partials (table j at partials + j n) added to *g_eps table
// by table, j = m-1 first: bitwise m launch_finalize calls in that order.
// sums: m doubles of scratch.
hipError_t launch_finalize_tables(const double* partials, int64_t n, int64_t m, double* sums,
                                  double* g_eps, hipStream_t st);

// Batched 2-D form.
struct BatchInst {
    int64_t offset;     // first element of the instance in the pool
    int nx, ny;
    Rates r;
};
struct BatchTile {
    int inst;           // instance index
    int x0, y0;         // tile origin
    int pad;            // multi-step tiles: end row of the segment
};
// rin / wout as for launch_step.
hipError_t launch_batch_step(const BatchInst* insts, const BatchTile* tiles, int64_t ntiles,
                             int tx, int ty, const double* src, double* dst, hipStream_t st,
                             bool rin = false, bool wout = false);
// nsteps (2, 4 or 8) steps per pass; tiles (inst, x0, y0, y1) cover strips of
// batch_strip_width(nsteps) columns (blocks of LW_THREADS threads).
constexpr int LW_THREADS = 128;
__host__ __device__ constexpr int batch_strip_width(int nsteps) { return LW_THREADS - 2 * nsteps; }
// off32: every instance's state is under 4 GiB (32-bit offsets from the
// instance's start).  one_wave: tiles are strips of strip_width(nsteps)
// columns run by the one-wave march of k_steps_d2q9; otherwise strips of
// batch_strip_width(nsteps) columns run by the two-wave LDS routine.
hipError_t launch_batch_steps(int nsteps, const BatchInst* insts, const BatchTile* tiles,
                              int64_t ntiles, const double* src, double* dst, bool off32,
                              bool one_wave, hipStream_t st, bool rin = false, bool wout = false);

}  // namespace lbm
