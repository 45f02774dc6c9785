// HIP kernels (gfx950) of the Cole-Hopf fourth-order MRT-LB solver.
//
// Data layout: a state buffer holds the q populations of every node in the
// chunked structure-of-arrays order of `slot` (lbm_kernels.h).  It is kept
// "stream-shifted": the slot of population i at node k holds f_i(k + e_i),
// the population that node k sent along e_i after its last collision, so one
// time step is a pull:
//     f_i(x) = src_i(x - e_i)          (pre-collision distribution at x)
//     dst_i(x) = (C f(x))_i            (collision, Sec. III.A)
// Every store is aligned and coalesced; the loads of a wavefront are 64
// consecutive doubles shifted by at most one element.  The update is
// HBM-bound (q*8 bytes read + q*8 written per node and step, a few flops per
// byte), so no matrix cores are used.
//
// Every thread owns one node; a block is 256 consecutive nodes of one row;
// y and (3-D) z run over grid.y and grid.z.
#include <atomic>
#include <type_traits>

#include "lbm_kernels.h"

namespace lbm {
namespace {

constexpr int BX = BLOCK_X;
constexpr int BY = BLOCK_Y;
constexpr int B1 = BLOCK_1D;

// Offsets of the neighbour x - e (e = -1, 0, +1) along each axis, periodic:
// s[a][e + 1] = ((x_a - e) mod n_a) * (stride of axis a in the node index).
struct Nbr {
    int s[4][3];
};

template <int D>
__device__ __forceinline__ Nbr make_nbr(const int (&c)[4], const Geo& g) {
    Nbr nb;
    const int n[4] = {g.nx, g.ny, g.nz, g.nw};
    int stride = 1;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (a < D) {
            const int m = c[a] == 0 ? n[a] - 1 : c[a] - 1;
            const int p = c[a] == n[a] - 1 ? 0 : c[a] + 1;
            nb.s[a][0] = p * stride;
            nb.s[a][1] = c[a] * stride;
            nb.s[a][2] = m * stride;
            stride *= n[a];
        } else {
            nb.s[a][0] = nb.s[a][1] = nb.s[a][2] = 0;
        }
    }
    return nb;
}

// Node index of x - e_i (pull source) and x + e_i (push target).
template <int D>
__device__ __forceinline__ int pull_index(const Nbr& nb, int i) {
    int k = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) k += nb.s[a][Lat<D>::E[i][a] + 1];
    return k;
}
template <int D>
__device__ __forceinline__ int push_index(const Nbr& nb, int i) {
    int k = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) k += nb.s[a][1 - Lat<D>::E[i][a]];
    return k;
}

__device__ __forceinline__ int64_t block_linear() {
    return (int64_t)blockIdx.x + (int64_t)gridDim.x * ((int64_t)blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip (linear
// block b runs on XCD b mod 8), each with its own L2.  Neighbouring tiles
// along x share the cache lines of the x +- 1 halo, so every XCD is given one
// contiguous range of tiles (x fastest) instead of every eighth tile.
constexpr unsigned NXCD = 8;
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb) {
    const unsigned q = nb / NXCD, r = nb % NXCD;
    const unsigned c = b % NXCD, slot = b / NXCD;
    return c * q + (c < r ? c : r) + slot;
}

template <int D>
__device__ __forceinline__ bool thread_node(const Geo& g, int (&c)[4]) {
    const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
    const unsigned b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const unsigned t = xcd_remap(b, nb);
    const unsigned tx = t % gridDim.x;
    const unsigned rest = t / gridDim.x;
    c[2] = c[3] = 0;
    if constexpr (D == 1) {
        c[0] = (int)(tx * B1 + threadIdx.x);
        c[1] = 0;
    } else {
        c[0] = (int)(tx * blockDim.x + threadIdx.x);
        c[1] = (int)((rest % gridDim.y) * blockDim.y + threadIdx.y);
        if constexpr (D >= 3) {
            const unsigned zw = rest / gridDim.y;  // grid.z runs over n_z * n_w
            if (D == 4 && (g.nz & 7) == 0 && (g.nw & 7) == 0) {
                // (z, w) planes in 8 x 8 patches, so that the blocks running
                // at the same time (about 64 planes of 64 x 64 nodes) hold
                // both the z and the w neighbours of most of their nodes in
                // L2: a twin is pulled from its partner's plane at the node
                // the partner's own pull does not read (64^4: +6 %)
                const unsigned p = zw >> 6, q = zw & 63, npz = (unsigned)g.nz >> 3;
                c[2] = (int)((p % npz) * 8 + (q & 7));
                c[3] = (int)((p / npz) * 8 + (q >> 3));
            } else {
                c[2] = (int)(zw % (unsigned)g.nz);
                c[3] = (int)(zw / (unsigned)g.nz);
            }
        }
    }
    return c[0] < g.nx && c[1] < g.ny;
}

__device__ __forceinline__ int node_index(const Geo& g, const int (&c)[4]) {
    return ((c[3] * g.nz + c[2]) * g.ny + c[1]) * g.nx + c[0];
}

// Deterministic sum over the 256 threads of a block; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    return tid == 0 ? (sh[0] + sh[1]) + (sh[2] + sh[3]) : 0.0;
}

// ---------------------------------------------------------------------------
// time step
// ---------------------------------------------------------------------------
// RIN: src was written by a collision, so a twin population is read from
// the plane of the population it equals (twin<D>); WOUT: the twins are not
// stored (dst then holds a state that only a RIN read may use).  Both leave
// the arithmetic, and so the result, bitwise unchanged.
template <int D, bool RIN = false, bool WOUT = false>
__global__ void __launch_bounds__(256) k_step(const double* __restrict__ src,
                                              double* __restrict__ dst, Geo g, Rates r) {
    constexpr int Q = Lat<D>::Q;
    int c[4];
    if (!thread_node<D>(g, c)) return;
    const Nbr nb = make_nbr<D>(c, g);
    double f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = src[slot<Q>(RIN ? twin<D>(i) : i, pull_index<D>(nb, i))];
    collide<D>(f, r);
    const int k = node_index(g, c);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        if (!WOUT || twin<D>(i) == i) __builtin_nontemporal_store(f[i], dst + slot<Q>(i, k));
}

// Small 1-D grids (n <= RESIDENT_MAX_1D): the whole state lives in LDS and
// one workgroup of T threads (PER nodes each, T * PER >= n) advances all
// nsteps in a single launch, so the run is not bound by one kernel launch per
// step; the smallest fitting shape keeps the per-step work and barrier cost
// proportional to n.  Same collision as k_step<1>.
//
// With walls != NULL the interval is bounded (wall_pull1): step s forms the
// distribution of the time whose boundary theta is wall_now (s = 0) or
// walls[2(s-1) .. 2(s-1)+1]; at the end wall_now takes the last pair.
// src and dst may be the same buffer (an even step count ends where it
// started): every load of src happens before the first store to dst, so the
// pointers carry no __restrict__.
template <int T, int PER>
__global__ void __launch_bounds__(T) k_step_resident1(const double* src, double* dst, int n,
                                                      int64_t nsteps, Rates r,
                                                      const double* __restrict__ walls,
                                                      double* __restrict__ wall_now) {
    constexpr int RES_THREADS = T;
    __shared__ double lds[3 * RESIDENT_MAX_1D];
    for (int x = threadIdx.x; x < n; x += RES_THREADS)
#pragma unroll
        for (int i = 0; i < 3; ++i) lds[i * RESIDENT_MAX_1D + x] = src[slot<3>(i, x)];
    __syncthreads();
    for (int64_t s = 0; s < nsteps; ++s) {
        const double* wall = walls ? (s == 0 ? wall_now : walls + 2 * (s - 1)) : nullptr;
        double f[PER][3];
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int x = threadIdx.x + p * RES_THREADS;
            if (x < n) {
                const int xm = x == 0 ? n - 1 : x - 1;
                const int xp = x == n - 1 ? 0 : x + 1;
                double g[3] = {lds[x], lds[RESIDENT_MAX_1D + xm], lds[2 * RESIDENT_MAX_1D + xp]};
                if (wall) {
                    if (x == 0) g[1] = wall[0] - (g[0] + g[2]);
                    if (x == n - 1) g[2] = wall[1] - (g[0] + g[1]);
                }
                collide<1>(g, r);
                f[p][0] = g[0];
                f[p][1] = g[1];
                f[p][2] = g[2];
            }
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int x = threadIdx.x + p * RES_THREADS;
            if (x < n) {
                lds[x] = f[p][0];
                lds[RESIDENT_MAX_1D + x] = f[p][1];
                lds[2 * RESIDENT_MAX_1D + x] = f[p][2];
            }
        }
        __syncthreads();
    }
    for (int x = threadIdx.x; x < n; x += RES_THREADS)
#pragma unroll
        for (int i = 0; i < 3; ++i) dst[slot<3>(i, x)] = lds[i * RESIDENT_MAX_1D + x];
    if (walls && nsteps > 0 && threadIdx.x < 2) wall_now[threadIdx.x] = walls[2 * (nsteps - 1) + threadIdx.x];
}

// ---------------------------------------------------------------------------
// 1-D interval with theta given at the end nodes (Example 1 of Sec. IV)
//
// Nodes x = 0..n-1 (n >= 2), the two ends on the boundary.  The distribution
// at x is pulled as usual, except for the one population that would come
// from outside the interval: it takes the value that makes sum_i f_i equal
// the boundary theta of the current time, wall[0] at x = 0 and wall[1] at
// x = n-1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wall_pull1(const double* __restrict__ src, int x, int n,
                                           const double* __restrict__ wall, double (&f)[3]) {
    f[0] = src[slot<3>(0, x)];
    f[1] = x > 0 ? src[slot<3>(1, x - 1)] : 0.0;
    f[2] = x < n - 1 ? src[slot<3>(2, x + 1)] : 0.0;
    if (x == 0) f[1] = wall[0] - (f[0] + f[2]);
    if (x == n - 1) f[2] = wall[1] - (f[0] + f[1]);
}

__global__ void __launch_bounds__(256) k_step_wall1(const double* __restrict__ src,
                                                    double* __restrict__ dst, int n, Rates r,
                                                    const double* __restrict__ wall) {
    const int x = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (x >= n) return;
    double f[3];
    wall_pull1(src, x, n, wall, f);
    collide<1>(f, r);
#pragma unroll
    for (int i = 0; i < 3; ++i) __builtin_nontemporal_store(f[i], dst + slot<3>(i, x));
}

// theta, u and grad theta as k_macro<1>, from the bounded-interval distribution.
__global__ void __launch_bounds__(256) k_macro_wall1(const double* __restrict__ src,
                                                     double* __restrict__ theta,
                                                     double* __restrict__ u,
                                                     double* __restrict__ grad, int n, Rates r,
                                                     const double* __restrict__ wall) {
    const int x = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (x >= n) return;
    double f[3];
    wall_pull1(src, x, n, wall, f);
    double th = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) th += f[i];
    if (theta) theta[x] = th;
    if (u || grad) {
        double j = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) j = LBM_SADD(j, Lat<1>::E[i][0], f[i]);
        if (u) u[x] = j * (r.ucoef / th);
        if (grad) grad[x] = r.gcoef * j;
    }
}

__global__ void __launch_bounds__(256) k_get_state_wall1(const double* __restrict__ src,
                                                         double* __restrict__ dense, int n,
                                                         const double* __restrict__ wall) {
    const int x = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (x >= n) return;
    double f[3];
    wall_pull1(src, x, n, wall, f);
#pragma unroll
    for (int i = 0; i < 3; ++i) dense[(int64_t)i * n + x] = f[i];
}

// Boundary theta of a dense 3 x n distribution: sum_i f_i at the end nodes.
__global__ void k_wall_from_dense1(const double* __restrict__ dense, int n, double* __restrict__ wall) {
    const int e = (int)threadIdx.x;
    if (e >= 2) return;
    const int x = e == 0 ? 0 : n - 1;
    wall[e] = (dense[x] + dense[(int64_t)n + x]) + dense[2 * (int64_t)n + x];
}

__device__ __forceinline__ int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// ---------------------------------------------------------------------------
// S D2Q9 time steps per pass over HBM (temporal blocking).
//
// One wave (64 lanes) owns a strip of 64 - 2S output columns plus an
// S-column halo on each side; lane t owns column x0 - S + t in every stage.
// The wave marches down a segment of rows: in iteration k it loads input
// row ys - S + k and stage j = 1..S computes row ys - S + k - j of step j from
// rows (that row + {-1, 0, +1}) of step j - 1.  Only stage S stores, so each
// value crosses HBM once per S steps (plus the halo).
//
// Exchange between stages never leaves the wave: a population with e_x = +1
// (-1) is pulled from the lane on the left (right) with a DPP wave shift
// (wave_shr:1 / wave_shl:1, two 32-bit moves per double), e_x = 0 stays in
// its lane.  Rows are delayed in registers: e_y = -1 is used in the
// iteration it arrives, e_y = 0 one iteration later, e_y = +1 two iterations
// later (two registers that alternate with the row parity; the march is
// unrolled by two so that the parity is static).  No LDS and no barrier.
//
// Every lane computes every stage (halo lanes produce values that only halo
// lanes consume); only stage S stores, from its valid lanes.  The first 2S
// iterations fill the pipeline (stage j holds valid rows from iteration 2j
// on) and are unrolled at compile time with the stages that are already
// valid, so the steady-state loop has no per-stage branch.  The arithmetic is
// collide<2> S times, so the result is bitwise that of S single steps.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int ms_ex(int i) { return Lat<2>::E[i][0]; }
__host__ __device__ constexpr int ms_ey(int i) { return Lat<2>::E[i][1]; }
// index of population i among those with the same e_y
__host__ __device__ constexpr int ms_yslot(int i) {
    int s = 0;
    for (int j = 0; j < i; ++j) s += ms_ey(j) == ms_ey(i);
    return s;
}

// value of a double in the lane on the left (DIR = +1) or right (DIR = -1)
template <int DIR>
__device__ __forceinline__ double lane_shift(double x) {
    constexpr int ctrl = DIR == 1 ? 0x138 : 0x130;  // wave_shr:1 : wave_shl:1
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), ctrl, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// value of a double in the lane on the left (DIR = +1) or right (DIR = -1),
// rotating around the wave (lane 0 takes lane 63 and vice versa)
template <int DIR>
__device__ __forceinline__ double lane_rotate(double x) {
    constexpr int ctrl = DIR == 1 ? 0x13C : 0x134;  // wave_ror:1 : wave_rol:1
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), ctrl, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// ---------------------------------------------------------------------------
// Small 1-D grids in one wave: lane l holds nodes l*PER .. l*PER+PER-1 in
// registers for the whole run; each step pulls f_{+1} from the node on the
// left and f_{-1} from the node on the right, inside the lane by register
// moves and across lanes by one DPP move each (a rotation for a periodic grid
// of exactly 64*PER nodes, a plain shift on a bounded interval, where the end
// nodes then take the wall rule of wall_pull1).  No LDS and no barrier; the
// arithmetic is that of k_step<1> / k_step_resident1.
// ---------------------------------------------------------------------------
// src and dst may be the same buffer, as for k_step_resident1.
template <int PER, bool PERIODIC>
__global__ void __launch_bounds__(64) k_step_wave1(const double* src, double* dst, int n,
                                                   int64_t nsteps,
                                                   Rates r, const double* __restrict__ walls,
                                                   double* __restrict__ wall_now) {
    const int lane = threadIdx.x;
    double s0[PER], sp[PER], sm[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int x = lane * PER + p;
        s0[p] = x < n ? src[slot<3>(0, x)] : 0.0;
        sp[p] = x < n ? src[slot<3>(1, x)] : 0.0;
        sm[p] = x < n ? src[slot<3>(2, x)] : 0.0;
    }
    for (int64_t s = 0; s < nsteps; ++s) {
        const double left = PERIODIC ? lane_rotate<1>(sp[PER - 1]) : lane_shift<1>(sp[PER - 1]);
        const double right = PERIODIC ? lane_rotate<-1>(sm[0]) : lane_shift<-1>(sm[0]);
        double w0 = 0.0, w1 = 0.0;
        if (!PERIODIC) {
            const double* wall = s == 0 ? wall_now : walls + 2 * (s - 1);
            w0 = wall[0];
            w1 = wall[1];
        }
        double t0[PER], tp[PER], tm[PER];
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int x = lane * PER + p;
            double g[3] = {s0[p], p > 0 ? sp[p - 1] : left, p < PER - 1 ? sm[p + 1] : right};
            if (!PERIODIC) {
                if (x == 0) g[1] = w0 - (g[0] + g[2]);
                if (x == n - 1) g[2] = w1 - (g[0] + g[1]);
            }
            collide<1>(g, r);
            t0[p] = g[0];
            tp[p] = g[1];
            tm[p] = g[2];
        }
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            s0[p] = t0[p];
            sp[p] = tp[p];
            sm[p] = tm[p];
        }
    }
#pragma unroll
    for (int p = 0; p < PER; ++p) {
        const int x = lane * PER + p;
        if (x < n) {
            dst[slot<3>(0, x)] = s0[p];
            dst[slot<3>(1, x)] = sp[p];
            dst[slot<3>(2, x)] = sm[p];
        }
    }
    if (!PERIODIC && nsteps > 0 && lane < 2) wall_now[lane] = walls[2 * (nsteps - 1) + lane];
}

// Addressing of a D2Q9 chunked buffer by node index k (population i at
// slot<9>(i, k)).  MsAddr<true>: the byte offset of population 0 as a 32-bit
// value from the buffer start, population i then at a base that is the same
// for the whole wave (buffer + i chunks), held in scalar registers; every
// access is one load or store with a scalar base and a 32-bit lane offset, and
// no 64-bit address arithmetic per access (the buffer must be under 4 GiB).
// MsAddr<false>: 64-bit element indices, any size.  Both address the same
// element, so the arithmetic and the results do not depend on the choice.
typedef __attribute__((address_space(1))) char GChar;
typedef __attribute__((address_space(1))) double GDouble;
__device__ __forceinline__ GChar* wave_base(const double* p) {
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (GChar*)(((unsigned long long)hi << 32) | lo);
}
template <bool OFF32> struct MsAddr;
typedef unsigned int MsU2 __attribute__((__vector_size__(8)));  // a double as buffer data
template <> struct MsAddr<true> {
    unsigned off;
    __device__ __forceinline__ explicit MsAddr(int k)
        : off((unsigned)((((k >> 12) * 9) << 12) | (k & (CHUNK - 1))) * 8u) {}
    __device__ __forceinline__ double load(const double* p, int i) const {
        return *(GDouble*)(wave_base(p + (int64_t)i * CHUNK) + off);
    }
    __device__ __forceinline__ void store(double* p, int i, double v) const {
        __builtin_nontemporal_store(v, (GDouble*)(wave_base(p + (int64_t)i * CHUNK) + off));
    }
    __device__ __forceinline__ void store_cached(double* p, int i, double v) const {
        *(GDouble*)(wave_base(p + (int64_t)i * CHUNK) + off) = v;
    }
};
template <> struct MsAddr<false> {
    int k;
    __device__ __forceinline__ explicit MsAddr(int k_) : k(k_) {}
    __device__ __forceinline__ double load(const double* p, int i) const { return p[slot<9>(i, k)]; }
    __device__ __forceinline__ void store(double* p, int i, double v) const {
        __builtin_nontemporal_store(v, p + slot<9>(i, k));
    }
    __device__ __forceinline__ void store_cached(double* p, int i, double v) const {
        p[slot<9>(i, k)] = v;
    }
};
// Whether a D2Q9 state buffer of g allows MsAddr<true>.
__host__ __device__ inline bool ms_off32(const Geo& g) {
    return (uint64_t)9 * (uint64_t)chunks_of(g.V) * CHUNK * sizeof(double) <= 0xffffffffull;
}

// Whether the plain D2Q9 passes write with cached stores: both state buffers
// fit in the 256 MB Infinity Cache, so the next pass finds its input there.
// Otherwise non-temporal stores are faster (8 steps per pass, GLUPS
// non-temporal / cached: 1024^2 196 / 207, 1280^2 216 / 247, 1448^2
// (288 MiB) 215 / 220, 1600^2 (352 MiB) 231 / 223, 4096^2 280 / 266).
constexpr uint64_t kInfinityCacheBytes = 256ull << 20;
inline bool d2q9_cached_stores(const Geo& g) {
    return 2ull * 9ull * (uint64_t)chunks_of(g.V) * CHUNK * sizeof(double) <= kInfinityCacheBytes;
}

template <int S>
struct MsState {
    double pre[9];      // next input row (prefetched)
    double z[S][3];     // e_y = 0 populations of the previous row, per stage input
    double u[2][S][3];  // e_y = +1 populations of the rows of each parity
};

// One iteration k of the march; P = k & 1; stages above ACTIVE are skipped
// (pipeline fill), stage S stores only when ACTIVE == S.  ALL: stage j < S
// also stores its rows of [ys, ye) to dst - (S - j) stride (the state after
// j steps, for a caller that keeps every intermediate state).  NT: stage S
// writes with non-temporal stores (otherwise through the caches).  UP: the
// march runs from row ye - 1 + S up to ys - S, so the roles of e_y = +1 and
// e_y = -1 in the row delays swap (same arithmetic per node).
template <int S, int P, int ACTIVE, bool ALL, bool OFF32, bool NT = true, bool RIN = false,
          bool WOUT = false, bool UP = false>
__device__ __forceinline__ void ms_row(MsState<S>& st, int k,
                                       const double* __restrict__ src, double* __restrict__ dst,
                                       int nx, int ny, int gx, int ys, int x0, const FoldedRates& r,
                                       int nrows, int64_t stride) {
    constexpr int W = MS_THREADS - 2 * S;
    const int lane = threadIdx.x;
    double f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = st.pre[RIN ? twin<2>(i) : i];
    {
        // Prefetch the next input row.  In the last iteration the row is not
        // used (its address is wrapped, so in bounds); loading it anyway
        // keeps the memory counters equal on both sides of the branch a
        // conditional load would need, so the wait at the row start is not
        // widened by a missing load (512^2: 90 -> 106 GLUPS).  The masked
        // stores of stage S still make that wait cover the previous row's
        // stores; two waves per SIMD hide it.
        const int row = UP ? ys + nrows - 1 + S - (k + 1) : ys - S + k + 1;
        const MsAddr<OFF32> a(wrapi(row, ny) * nx + gx);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            if (!RIN || twin<2>(i) == i) st.pre[i] = a.load(src, i);
    }
#pragma unroll
    for (int j = 1; j <= S; ++j) {
        // inputs of stage j: stage j-1 rows of iterations k (e_y = -1), k-1
        // (e_y = 0) and k-2 (e_y = +1), pulled from lane t - e_x (marching
        // up, e_y = +1 and -1 trade places)
        double in[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double v = ms_ex(i) == 0 ? f[i]
                                           : (ms_ex(i) == 1 ? lane_shift<1>(f[i]) : lane_shift<-1>(f[i]));
            const int ey = UP ? -ms_ey(i) : ms_ey(i);
            if (ey == -1) {
                in[i] = v;
            } else if (ey == 0) {
                in[i] = st.z[j - 1][ms_yslot(i)];
                st.z[j - 1][ms_yslot(i)] = v;
            } else {
                in[i] = st.u[P][j - 1][ms_yslot(i)];
                st.u[P][j - 1][ms_yslot(i)] = v;
            }
        }
        if (j <= ACTIVE) {
            collide_d2q9(in, r);
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = in[i];
            if (j == S && ACTIVE == S && lane >= S && lane < S + W && x0 - S + lane < nx) {
                const int row = UP ? ys + nrows - 1 + 2 * S - k : ys - 2 * S + k;
                const MsAddr<OFF32> a(wrapi(row, ny) * nx + x0 - S + lane);
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    if (WOUT && twin<2>(i) != i) continue;
                    if constexpr (NT)
                        a.store(dst, i, in[i]);
                    else
                        a.store_cached(dst, i, in[i]);
                }
            }
            if (ALL && j < S) {
                // row ys + k - S - j of step j; lanes S .. S+W-1 hold valid
                // values from stage j on (the valid band shrinks one lane per
                // side per stage)
                const int rr = k - S - j;
                if (rr >= 0 && rr < nrows && lane >= S && lane < S + W && x0 - S + lane < nx) {
                    const MsAddr<OFF32> a((UP ? ys + nrows - 1 - rr : ys + rr) * nx + x0 - S + lane);
                    double* out = dst - (int64_t)(S - j) * stride;
                    if constexpr (OFF32) {
                        // a buffer descriptor per state and the plane as a
                        // scalar offset shared by all S states: a 64-bit
                        // base per plane and state would exceed the scalar
                        // registers (they spill into VGPR lanes).  Records:
                        // the bytes of one state (below 2^32 here); cache
                        // policy 2 is the non-temporal hint of the other
                        // stores.
                        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                            out, (short)0, (int)(unsigned)((uint64_t)9 * CHUNK * 8 *
                                                          (uint64_t)((nx * ny + CHUNK - 1) >> 12)),
                            0x00020000);
#pragma unroll
                        for (int i = 0; i < 9; ++i)
                            if (!WOUT || twin<2>(i) == i)
                                __builtin_amdgcn_raw_buffer_store_b64(
                                    __builtin_bit_cast(MsU2, in[i]), rs, a.off, i * CHUNK * 8, 2);
                    } else {
#pragma unroll
                        for (int i = 0; i < 9; ++i)
                            if (!WOUT || twin<2>(i) == i) a.store(out, i, in[i]);
                    }
                }
            }
        }
    }
}

template <int S, int K, bool ALL, bool OFF32, bool NT = true, bool RIN = false, bool WOUT = false,
          bool UP = false>
__device__ __forceinline__ void ms_fill(MsState<S>& st, const double* __restrict__ src,
                                        double* __restrict__ dst, int nx, int ny, int gx, int ys,
                                        int x0, const FoldedRates& r, int nrows, int64_t stride) {
    if constexpr (K < 2 * S) {
        ms_row<S, K & 1, K / 2, ALL, OFF32, NT, RIN, WOUT, UP>(st, K, src, dst, nx, ny, gx, ys, x0,
                                                               r, nrows, stride);
        ms_fill<S, K + 1, ALL, OFF32, NT, RIN, WOUT, UP>(st, src, dst, nx, ny, gx, ys, x0, r, nrows,
                                                         stride);
    }
}

// Advance rows [ys, ye) (ye > ys) of the columns [x0, x0 + 64 - 2S) of one
// D2Q9 grid by S steps (reads rows ys-S .. ye-1+S and columns x0-S ..
// x0+63-S, wrapped periodically), marching down the rows or, with UP, up.
// All 64 lanes of the wave must be active.
template <int S, bool ALL, bool OFF32, bool NT = true, bool RIN = false, bool WOUT = false,
          bool UP = false>
__device__ __forceinline__ void ms_tile(const double* __restrict__ src, double* __restrict__ dst,
                                        int nx, int ny, const FoldedRates& r, int x0, int ys,
                                        int ye, int64_t stride = 0) {
    const int gx = wrapi(x0 - S + (int)threadIdx.x, nx);
    const int kend = ye - ys + 2 * S - 1;  // >= 2S
    MsState<S> st;
    {
        const MsAddr<OFF32> a(wrapi(UP ? ye - 1 + S : ys - S, ny) * nx + gx);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            if (!RIN || twin<2>(i) == i) st.pre[i] = a.load(src, i);
    }
#pragma unroll
    for (int j = 0; j < S; ++j)
#pragma unroll
        for (int a = 0; a < 3; ++a) st.z[j][a] = st.u[0][j][a] = st.u[1][j][a] = 0.0;
    const int nrows = ye - ys;
    ms_fill<S, 0, ALL, OFF32, NT, RIN, WOUT, UP>(st, src, dst, nx, ny, gx, ys, x0, r, nrows,
                                                 stride);
    // whole row pairs in the loop and a last odd row after it: the loop then
    // has a single path back to its head, and the compiler keeps the row
    // delays in place instead of copying them at the join (bitwise the same;
    // 37 instead of 52 copies per row pair)
    int k = 2 * S;
    for (; k + 1 <= kend; k += 2) {
        ms_row<S, 0, S, ALL, OFF32, NT, RIN, WOUT, UP>(st, k, src, dst, nx, ny, gx, ys, x0, r,
                                                       nrows, stride);
        ms_row<S, 1, S, ALL, OFF32, NT, RIN, WOUT, UP>(st, k + 1, src, dst, nx, ny, gx, ys, x0, r,
                                                       nrows, stride);
    }
    if (k <= kend)
        ms_row<S, 0, S, ALL, OFF32, NT, RIN, WOUT, UP>(st, k, src, dst, nx, ny, gx, ys, x0, r,
                                                       nrows, stride);
}

// Two waves per SIMD: the register budget (256 per wave) holds S = 8.
// RIN / WOUT: twin populations read from their twins' planes / not stored,
// as for k_step.  Odd row segments march up: two neighbouring segments then
// read the halo rows they share at the same time (both at their ends, or
// both at their starts), so the second read finds them in the caches
// (512^2 +2.7 %, 1024^2 +1.3 %, 2048^2 +1.7 %, 4096^2 +0.7 %).
template <int S, bool OFF32, bool RIN, bool WOUT>
__global__ void __launch_bounds__(MS_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
k_steps_d2q9(const double* __restrict__ src,
                                                           double* __restrict__ dst, Geo g,
                                                           Rates r, int ly, int nstrips) {
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int strip = (int)(t % (unsigned)nstrips);
    const int seg = (int)(t / (unsigned)nstrips);
    const int ys = seg * ly;
    if (seg & 1)
        ms_tile<S, false, OFF32, true, RIN, WOUT, true>(src, dst, g.nx, g.ny, folded(r),
                                                        strip * strip_width(S), ys,
                                                        min(ys + ly, g.ny), 0);
    else
        ms_tile<S, false, OFF32, true, RIN, WOUT>(src, dst, g.nx, g.ny, folded(r),
                                                  strip * strip_width(S), ys, min(ys + ly, g.ny),
                                                  0);
}

// The same pass with cached stores, for grids whose two states fit in the
// Infinity Cache (the next pass then reads its input from there).
template <int S, bool OFF32, bool RIN, bool WOUT>
__global__ void __launch_bounds__(MS_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
k_steps_d2q9_cached(const double* __restrict__ src, double* __restrict__ dst, Geo g, Rates r,
                    int ly, int nstrips) {
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int strip = (int)(t % (unsigned)nstrips);
    const int seg = (int)(t / (unsigned)nstrips);
    const int ys = seg * ly;
    if (seg & 1)
        ms_tile<S, false, OFF32, false, RIN, WOUT, true>(src, dst, g.nx, g.ny, folded(r),
                                                         strip * strip_width(S), ys,
                                                         min(ys + ly, g.ny), 0);
    else
        ms_tile<S, false, OFF32, false, RIN, WOUT>(src, dst, g.nx, g.ny, folded(r),
                                                   strip * strip_width(S), ys,
                                                   min(ys + ly, g.ny), 0);
}

// The same pass writing the state after every one of its S steps: step j to
// out + (j - 1) stride (the adjoint's recomputation of a checkpoint segment).
// RIN / WOUT as for k_step (WOUT applies to every state written).
template <int S, bool OFF32, bool RIN, bool WOUT>
__global__ void __launch_bounds__(MS_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
k_steps_d2q9_all(const double* __restrict__ src, double* __restrict__ out, int64_t stride, Geo g,
                 Rates r, int ly, int nstrips) {
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int strip = (int)(t % (unsigned)nstrips);
    const int seg = (int)(t / (unsigned)nstrips);
    const int ys = seg * ly;
    ms_tile<S, true, OFF32, true, RIN, WOUT>(src, out + (int64_t)(S - 1) * stride, g.nx, g.ny,
                                             folded(r), strip * strip_width(S), ys,
                                             min(ys + ly, g.ny), stride);
}

// ---------------------------------------------------------------------------
// S adjoint D2Q9 steps per pass (the reverse sweep of a checkpoint segment).
//
// An adjoint step maps lambda^{n+1} to lambda^n = C^T mu with
// mu_i(x) = lambda^{n+1}_i(x + e_i): the forward step with every velocity
// reversed and C^T in place of C.  The one-wave march of k_steps_d2q9 applies
// with e -> -e (a population with e_y = +1 is used in the iteration its row
// arrives, e_y = -1 two iterations later; e_x = +1 comes from the lane on the
// right).  Stage j produces lambda^{N-j} from lambda^{N-j+1}; at the nodes the
// wave owns it also adds the eps part <mu, (dC/deps) f^{N-j}> (through the
// dual moments of mu, eps_part_d2q9), with f^{N-j}
// pulled from its state buffer at ftop - (j - 1) stride (ftop = f^{N-1});
// RIN: those states were written by a collision and twin populations are
// read from their partners' planes (as in k_step).  The partner planes of the
// twins (those of the (+,+) and (-,+) edges) serve two rows of the pull each
// (row y - 1 for the edge itself, row y + 1 for its twin), so each of their
// rows is loaded once at the lane's own column, kept two rows in a per-wave
// LDS delay and pulled along x by a DPP lane shift (as_load_f_tw, as_edges):
// every plane row of the recomputed states is read once per pass.
// Each lane sums the eps parts of its nodes over all stages and rows in a
// fixed order; the wave's sum goes to partials[block], and the blocks from
// nblocks to ntab - 1 write zeros, so the table always holds ntab entries.
// lambda is bitwise that of S launches of k_adjoint_step<2>.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int as_ex(int i) { return -Lat<2>::E[i][0]; }
__host__ __device__ constexpr int as_ey(int i) { return -Lat<2>::E[i][1]; }

template <int S>
struct AsState : MsState<S> {
    double fp[S][9];  // f^{N-j} at the node of the next iteration's row, per stage
};

// f^{N-j} pulled at node (x, y): population i from (x - e_i, y - e_i).
template <bool RIN>
__device__ __forceinline__ void as_load_f(double (&fn)[9], const double* __restrict__ fs, int x,
                                          int y, int nx, int ny) {
    const int rows[3] = {wrapi(y + 1, ny) * nx, y * nx, wrapi(y - 1, ny) * nx};
    const int cols[3] = {x == nx - 1 ? 0 : x + 1, x, x == 0 ? nx - 1 : x - 1};
#pragma unroll
    for (int i = 0; i < 9; ++i)
        fn[i] = fs[slot<9>(RIN ? twin<2>(i) : i, rows[ms_ey(i) + 1] + cols[ms_ex(i) + 1])];
}

// RIN: the per-wave LDS delay of the two partner planes for stage j holds,
// per row parity, the raw rows (own column of each lane) of planes 5 and 6:
// tw[((j - 1) * 2 + parity) * 128 + plane * 64 + lane].  Each lane reads
// and writes only its own entries.
constexpr int AS_TW = 128;  // doubles per stage and parity
// f^{N-j} for row y (RIN): populations 0-4 pulled as in as_load_f (own
// lanes); fn[7], fn[8] the raw rows y + 1 of planes 5 and 6 (every lane).
// as_edges completes the pull when the row is used.
__device__ __forceinline__ void as_load_f_tw(double (&fn)[9], const double* __restrict__ fs,
                                             int x, int gx, int y, int nx, int ny, bool own) {
    if (own) {
        const int rows[3] = {wrapi(y + 1, ny) * nx, y * nx, wrapi(y - 1, ny) * nx};
        const int cols[3] = {x == nx - 1 ? 0 : x + 1, x, x == 0 ? nx - 1 : x - 1};
#pragma unroll
        for (int i = 0; i < 5; ++i) fn[i] = fs[slot<9>(i, rows[ms_ey(i) + 1] + cols[ms_ex(i) + 1])];
    }
    const int yp = wrapi(y + 1, ny) * nx + gx;
    fn[7] = fs[slot<9>(5, yp)];
    fn[8] = fs[slot<9>(6, yp)];
}
// Row y of stage j: take the raw rows y - 1 of planes 5 and 6 from the LDS
// delay (stored two rows earlier, or at the start of the segment), store the
// raw rows y + 1 in their place for row y + 2, and pull the four edge
// populations along x: population i of plane 5 or 6 from the lane at
// x - e_x (e = (1,1), (-1,1) from row y - 1; (-1,-1), (1,-1) from row y + 1).
__device__ __forceinline__ void as_edges(double (&fn)[9], double* tw) {
    const double m5 = tw[threadIdx.x], m6 = tw[64 + threadIdx.x];
    tw[threadIdx.x] = fn[7];
    tw[64 + threadIdx.x] = fn[8];
    fn[5] = lane_shift<1>(m5);
    fn[6] = lane_shift<-1>(m6);
    fn[7] = lane_shift<-1>(fn[7]);
    fn[8] = lane_shift<1>(fn[8]);
}
static_assert(ms_ex(5) == 1 && ms_ey(5) == 1 && ms_ex(6) == -1 && ms_ey(6) == 1 &&
                  twin<2>(7) == 5 && twin<2>(8) == 6,
              "the edge planes 5 and 6 carry the (+,+) and (-,+) edges and their twins");

template <int S, int P, int ACTIVE, bool RIN>
__device__ __forceinline__ void as_row(AsState<S>& st, double& ge, int k,
                                       const double* __restrict__ src, double* __restrict__ dst,
                                       const double* __restrict__ ftop, int64_t stride, int nx,
                                       int ny, int gx, int ys, int x0, int nrows, const Rates& r,
                                       double* tw) {
    constexpr int W = MS_THREADS - 2 * S;
    const int lane = threadIdx.x;
    const int x = x0 - S + lane;
    const bool own = lane >= S && lane < S + W && x < nx;
    double f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = st.pre[i];
    {
        // next lambda row (unused in the last iteration, as in ms_row)
        const int base = wrapi(ys - S + k + 1, ny) * nx + gx;
#pragma unroll
        for (int i = 0; i < 9; ++i) st.pre[i] = src[slot<9>(i, base)];
    }
#pragma unroll
    for (int j = 1; j <= S; ++j) {
        double in[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double v = as_ex(i) == 0 ? f[i]
                                           : (as_ex(i) == 1 ? lane_shift<1>(f[i]) : lane_shift<-1>(f[i]));
            if (as_ey(i) == -1) {
                in[i] = v;
            } else if (as_ey(i) == 0) {
                in[i] = st.z[j - 1][ms_yslot(i)];
                st.z[j - 1][ms_yslot(i)] = v;
            } else {
                in[i] = st.u[P][j - 1][ms_yslot(i)];
                st.u[P][j - 1][ms_yslot(i)] = v;
            }
        }
        if (j <= ACTIVE) {
            const int rr = k - S - j;  // owned row ys + rr of this stage
            // the dual moments of mu serve the eps part and C^T mu
            const Dual2 du = dual_d2q9(in);
            if (rr >= 0 && rr < nrows) {
                if constexpr (RIN) as_edges(st.fp[j - 1], tw + ((j - 1) * 2 + (rr & 1)) * AS_TW);
                if (own) ge += eps_part_d2q9(du, st.fp[j - 1], r);
            }
            double lam[9];
            collide_adjoint_d2q9(du, r, lam);  // as collide_adjoint<2>
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = lam[i];
            if (j == S && ACTIVE == S && own) {
                const int row = (ys + k - 2 * S) * nx + x;
#pragma unroll
                for (int i = 0; i < 9; ++i) dst[slot<9>(i, row)] = lam[i];
            }
        }
    }
    // f^{N-j} for the rows the stages own in the next iteration
#pragma unroll
    for (int j = 1; j <= S; ++j) {
        const int rr = k + 1 - S - j;
        if constexpr (RIN) {
            if (rr >= 0 && rr < nrows)
                as_load_f_tw(st.fp[j - 1], ftop - (int64_t)(j - 1) * stride, x, gx, ys + rr, nx,
                             ny, own);
        } else {
            if (own && rr >= 0 && rr < nrows)
                as_load_f<RIN>(st.fp[j - 1], ftop - (int64_t)(j - 1) * stride, x, ys + rr, nx, ny);
        }
    }
}

template <int S, int K, bool RIN>
__device__ __forceinline__ void as_fill(AsState<S>& st, double& ge,
                                        const double* __restrict__ src, double* __restrict__ dst,
                                        const double* __restrict__ ftop, int64_t stride, int nx,
                                        int ny, int gx, int ys, int x0, int nrows, const Rates& r,
                                        double* tw) {
    if constexpr (K < 2 * S) {
        as_row<S, K & 1, K / 2, RIN>(st, ge, K, src, dst, ftop, stride, nx, ny, gx, ys, x0, nrows,
                                     r, tw);
        as_fill<S, K + 1, RIN>(st, ge, src, dst, ftop, stride, nx, ny, gx, ys, x0, nrows, r, tw);
    }
}

template <int S, bool RIN>
__global__ void __launch_bounds__(MS_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
k_adjoint_steps_d2q9(const double* __restrict__ src, double* __restrict__ dst,
                     const double* __restrict__ ftop, int64_t stride,
                     double* __restrict__ partials, int ntab, Geo g, Rates r, int ly,
                     int nstrips) {
    const int nx = g.nx, ny = g.ny;
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const int strip = (int)(t % (unsigned)nstrips);
    const int seg = (int)(t / (unsigned)nstrips);
    const int x0 = strip * strip_width(S);
    const int ys = seg * ly;
    const int ye = min(ys + ly, ny);
    const int gx = wrapi(x0 - S + (int)threadIdx.x, nx);
    const int kend = ye - ys + 2 * S - 1;
    const int nrows = ye - ys;
    AsState<S> st;
    {
        const int base = wrapi(ys - S, ny) * nx + gx;
#pragma unroll
        for (int i = 0; i < 9; ++i) st.pre[i] = src[slot<9>(i, base)];
    }
#pragma unroll
    for (int j = 0; j < S; ++j) {
#pragma unroll
        for (int a = 0; a < 3; ++a) st.z[j][a] = st.u[0][j][a] = st.u[1][j][a] = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) st.fp[j][i] = 0.0;
    }
    // RIN: the LDS delay of the partner planes starts with the raw rows
    // ys - 1 (parity 0) and ys (parity 1) of every stage's state; each lane
    // reads back only what it wrote, so no barrier is needed
    __shared__ double tw[RIN ? S * 2 * AS_TW : 1];
    if constexpr (RIN) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const double* fs = ftop - (int64_t)j * stride;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int row = wrapi(ys - 1 + p, ny) * nx + gx;
                tw[(j * 2 + p) * AS_TW + threadIdx.x] = fs[slot<9>(5, row)];
                tw[(j * 2 + p) * AS_TW + 64 + threadIdx.x] = fs[slot<9>(6, row)];
            }
        }
    }
    double ge = 0.0;
    as_fill<S, 0, RIN>(st, ge, src, dst, ftop, stride, nx, ny, gx, ys, x0, nrows, r, tw);
    // row pairs in the loop, a last odd row after it (as in ms_tile)
    int k = 2 * S;
    for (; k + 1 <= kend; k += 2) {
        as_row<S, 0, S, RIN>(st, ge, k, src, dst, ftop, stride, nx, ny, gx, ys, x0, nrows, r, tw);
        as_row<S, 1, S, RIN>(st, ge, k + 1, src, dst, ftop, stride, nx, ny, gx, ys, x0, nrows, r,
                             tw);
    }
    if (k <= kend)
        as_row<S, 0, S, RIN>(st, ge, k, src, dst, ftop, stride, nx, ny, gx, ys, x0, nrows, r, tw);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ge += __shfl_xor(ge, o, 64);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = ge;
        for (int i = (int)gridDim.x + (int)blockIdx.x; i < ntab; i += (int)gridDim.x)
            partials[i] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// S D3Q19 time steps per pass over HBM.
//
// The 2-D scheme above one dimension up: a block of MS3_TX x MS3_TY threads
// owns a tile of (MS3_TX - 2S) x (MS3_TY - 2S) output columns (x, y) plus an
// S-wide halo, thread (tx, ty) owns one column in every stage, and the block
// marches along z through a segment of planes.  A row of the tile (fixed y)
// is one wave, lane tx = column x: the ten populations with e_x != 0 are
// pulled from lane tx - e_x by DPP lane shifts, as in the D2Q9 passes; the
// ten with e_y != 0 (the xy edges after their x shift) then go through LDS
// to row ty + e_y; the three with e_x = e_y = 0 stay in their thread.  Planes
// are delayed in registers by e_z (0, 1 or 2 iterations).  Register pressure
// limits S to 2 (190 VGPRs when only the 13 independent populations are
// loaded, 217 otherwise; two waves per SIMD, so one 512-thread block per
// CU); each block uses 2 x 10 x 512 doubles of LDS.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int m3_ex(int i) { return Lat<3>::E[i][0]; }
__host__ __device__ constexpr int m3_ey(int i) { return Lat<3>::E[i][1]; }
__host__ __device__ constexpr int m3_ez(int i) { return Lat<3>::E[i][2]; }
// index of population i among those with its e_z
__host__ __device__ constexpr int m3_zslot(int i) {
    int s = 0;
    for (int j = 0; j < i; ++j) s += m3_ez(j) == m3_ez(i);
    return s;
}
constexpr int M3_Z0 = 9, M3_ZP = 5;  // populations with e_z = 0 and with e_z = +1
constexpr int M3_THREADS = MS3_TX * MS3_TY;
static_assert(MS3_TX == 64, "a tile row of the D3Q19 pass is one wave (DPP lane shifts along x)");

template <int S>
struct Ms3State {
    double pre[19];            // next input plane (prefetched)
    double z[S][M3_Z0];        // e_z = 0 populations of the previous plane, per stage input
    double u[2][S][M3_ZP];     // e_z = +1 populations of the planes of each parity
};

// y-movers (e_y != 0): the 10 populations exchanged through LDS
__host__ __device__ constexpr bool m3_ymover(int i) { return m3_ey(i) != 0; }
__host__ __device__ constexpr int m3_yslot(int i) {
    int s = 0;
    for (int j = 0; j < i; ++j) s += m3_ymover(j);
    return s;
}
constexpr int M3_YMOVERS = m3_yslot(19);
static_assert(M3_YMOVERS == 10, "D3Q19 has 10 populations with e_y != 0");

// Whether plane i of a post-collision state (population i, or its twin)
// holds a population with e_y = ey.
__host__ __device__ constexpr bool m3_plane_holds(int i, int ey) {
    for (int p = 0; p < 19; ++p)
        if (twin<3>(p) == i && m3_ey(p) == ey) return true;
    return false;
}
__host__ __device__ constexpr int m3_planes_holding(int ey) {
    int n = 0;
    for (int i = 0; i < 19; ++i) n += twin<3>(i) == i && m3_plane_holds(i, ey);
    return n;
}
static_assert(m3_planes_holding(1) == 5 && m3_planes_holding(-1) == 5,
              "an edge row of the tile passes on 5 of the 13 independent planes");

// With only the 13 independent populations, one input plane (z-plane zp) of
// the column col through a buffer resource over that z-plane's chunks
// (32-bit offsets).  The first tile row passes on only its populations with
// e_y = +1 and the last only those with e_y = -1; the planes they do not
// need get an out-of-range offset, so the hardware drops those loads (no
// memory access, the register reads 0) and every wave still issues the same
// instructions: the two edge rows fetch 5 of the 13 planes.
__device__ __forceinline__ void m3_load_plane(double (&pre)[19], const double* src,
                                              int64_t plane, int zp, int col, int ty) {
    const int64_t n0 = (int64_t)zp * plane;
    const int64_t c0 = n0 >> 12, c1 = (n0 + plane - 1) >> 12;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double*>(src) + c0 * 19 * 4096, (short)0,
        (int)((c1 - c0 + 1) * 19 * 4096 * 8), 0x00020000);
    const int64_t kk = n0 + col;
    const unsigned base = (unsigned)((((kk >> 12) - c0) * 19 * 4096 + (kk & 4095)) * 8);
#pragma unroll
    for (int i = 0; i < 19; ++i)
        if (twin<3>(i) == i) {
            const bool need = (ty != 0 || m3_plane_holds(i, 1)) &&
                              (ty != MS3_TY - 1 || m3_plane_holds(i, -1));
            const unsigned off = need ? base + (unsigned)(i * 4096 * 8) : 0x80000000u;
            pre[i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
        }
}

// x shift by DPP (pull from lane tx - e_x), then y shift through LDS.  BUF:
// the input planes come through m3_load_plane (RIN only).
template <int S, int P, bool RIN, bool WOUT, bool BUF = false>
__device__ __forceinline__ void ms3_plane(Ms3State<S>& st, double* lds, int k,
                                          const double* __restrict__ src, double* __restrict__ dst,
                                          const Geo& g, int col, int zs, int x0, int y0,
                                          const FoldedRates& r) {
    static_assert(!BUF || RIN, "buffer loads serve the reduced state only");
    // a tile row is one wave: ty is uniform across it, and saying so lets the
    // per-row choices (edge-row loads, y exchange) compile to scalar selects
    // and branches instead of lane-masked ones
    const int tid = threadIdx.x, tx = tid % MS3_TX;
    const int ty = __builtin_amdgcn_readfirstlane(tid / MS3_TX);
    const int64_t plane = (int64_t)g.nx * g.ny;
    double f[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) f[i] = st.pre[RIN ? twin<3>(i) : i];
    if constexpr (BUF) {
        m3_load_plane(st.pre, src, plane, wrapi(zs - S + k + 1, g.nz), col, ty);
    } else {
        const int64_t base = (int64_t)wrapi(zs - S + k + 1, g.nz) * plane + col;
#pragma unroll
        for (int i = 0; i < 19; ++i)
            if (!RIN || twin<3>(i) == i) st.pre[i] = src[slot<19>(i, base)];
    }
    // pull along x (every lane takes part; the edge lanes receive zeros,
    // which reach only halo columns, never a stored output)
#pragma unroll
    for (int i = 0; i < 19; ++i)
        if (m3_ex(i) != 0) f[i] = m3_ex(i) == 1 ? lane_shift<1>(f[i]) : lane_shift<-1>(f[i]);
#pragma unroll
    for (int i = 0; i < 19; ++i)
        if (m3_ymover(i)) {
            const int cy = ty + m3_ey(i);
            if (cy >= 0 && cy < MS3_TY) lds[m3_yslot(i) * M3_THREADS + cy * MS3_TX + tx] = f[i];
        }
    __syncthreads();
#pragma unroll
    for (int j = 1; j <= S; ++j) {
        double in[19];
        const double* rd = lds + ((j - 1) & 1) * M3_YMOVERS * M3_THREADS;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            const double v = m3_ymover(i) ? rd[m3_yslot(i) * M3_THREADS + tid] : f[i];
            if (m3_ez(i) == -1) {
                in[i] = v;
            } else if (m3_ez(i) == 0) {
                in[i] = st.z[j - 1][m3_zslot(i)];
                st.z[j - 1][m3_zslot(i)] = v;
            } else {
                in[i] = st.u[P][j - 1][m3_zslot(i)];
                st.u[P][j - 1][m3_zslot(i)] = v;
            }
        }
        if (k >= 2 * j) {
            collide_d3q19(in, r);
            if (j < S) {
                double* wr = lds + (j & 1) * M3_YMOVERS * M3_THREADS;
#pragma unroll
                for (int i = 0; i < 19; ++i) {
                    double v = in[i];
                    if (m3_ex(i) != 0) v = m3_ex(i) == 1 ? lane_shift<1>(v) : lane_shift<-1>(v);
                    f[i] = v;
                    if (m3_ymover(i)) {
                        const int cy = ty + m3_ey(i);
                        if (cy >= 0 && cy < MS3_TY) wr[m3_yslot(i) * M3_THREADS + cy * MS3_TX + tx] = v;
                    }
                }
            } else if (tx >= S && tx < MS3_TX - S && ty >= S && ty < MS3_TY - S &&
                       x0 - S + tx < g.nx && y0 - S + ty < g.ny) {
                const int64_t kk = (int64_t)wrapi(zs - 2 * S + k, g.nz) * plane +
                                   (int64_t)(y0 - S + ty) * g.nx + (x0 - S + tx);
#pragma unroll
                for (int i = 0; i < 19; ++i)
                    if (!WOUT || twin<3>(i) == i)
                        __builtin_nontemporal_store(in[i], dst + slot<19>(i, kk));
            }
        }
        if (j < S) __syncthreads();
    }
    if (S & 1) __syncthreads();
}

template <int S, bool RIN, bool WOUT, bool BUF>
__global__ void __launch_bounds__(M3_THREADS) k_steps_d3q19(const double* __restrict__ src,
                                                            double* __restrict__ dst, Geo g,
                                                            Rates r, int lz, int ntx, int nty) {
    __shared__ double lds[2 * M3_YMOVERS * M3_THREADS];
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    const unsigned ntile = (unsigned)ntx * (unsigned)nty;
    const int tile = (int)(t % ntile), seg = (int)(t / ntile);
    const int x0 = (tile % ntx) * tile_width3(S), y0 = (tile / ntx) * tile_height3(S);
    const int zs = seg * lz, ze = min(zs + lz, g.nz);
    const int tx = threadIdx.x % MS3_TX;
    const int ty = __builtin_amdgcn_readfirstlane((int)threadIdx.x / MS3_TX);
    const int col = wrapi(y0 - S + ty, g.ny) * g.nx + wrapi(x0 - S + tx, g.nx);
    const int kend = ze - zs + 2 * S - 1;
    const FoldedRates fr = folded(r);
    Ms3State<S> st;
    {
        const int64_t base = (int64_t)wrapi(zs - S, g.nz) * g.nx * g.ny + col;
#pragma unroll
        for (int i = 0; i < 19; ++i)
            if (!RIN || twin<3>(i) == i) st.pre[i] = src[slot<19>(i, base)];
    }
#pragma unroll
    for (int j = 0; j < S; ++j) {
#pragma unroll
        for (int a = 0; a < M3_Z0; ++a) st.z[j][a] = 0.0;
#pragma unroll
        for (int a = 0; a < M3_ZP; ++a) st.u[0][j][a] = st.u[1][j][a] = 0.0;
    }
    // plane pairs in the loop, a last odd plane after it (as in ms_tile)
    int k = 0;
    for (; k + 1 <= kend; k += 2) {
        ms3_plane<S, 0, RIN, WOUT, BUF>(st, lds, k, src, dst, g, col, zs, x0, y0, fr);
        ms3_plane<S, 1, RIN, WOUT, BUF>(st, lds, k + 1, src, dst, g, col, zs, x0, y0, fr);
    }
    if (k <= kend) ms3_plane<S, 0, RIN, WOUT, BUF>(st, lds, k, src, dst, g, col, zs, x0, y0, fr);
}

// ---------------------------------------------------------------------------
// initialisation
// ---------------------------------------------------------------------------
// Fourth-order central difference of theta along axis a at node c.
template <int D>
__device__ double fd4(const double* __restrict__ th, const Geo& g, const int (&c)[4], int a,
                      double inv12dx) {
    const int n[4] = {g.nx, g.ny, g.nz, g.nw};
    double v[4];
    const int off[4] = {2, 1, -1, -2};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        int cc[4] = {c[0], c[1], c[2], c[3]};
        cc[a] = wrapi(c[a] + off[t], n[a]);
        v[t] = th[node_index(g, cc)];
    }
    return ((v[3] - v[0]) + 8.0 * (v[1] - v[2])) * inv12dx;
}

// dst_i(y) = f0_i(y + e_i) with the closed-form initial distribution
// f0_i = w_i theta0 - dx w_i (e_i . g) - (1/s1 - 1)(dx/6) sum_a (d_{i,+a} - d_{i,-a}) g_a.
template <int D>
__global__ void __launch_bounds__(256) k_init(const double* __restrict__ th0,
                                              const double* __restrict__ grad,
                                              double* __restrict__ dst, Geo g, Rates r) {
    constexpr int Q = Lat<D>::Q;
    int c[4];
    if (!thread_node<D>(g, c)) return;
    const int k = node_index(g, c);
    const double corr = r.inv_s1_m1 * r.dx * (1.0 / 6.0);
    const int n[4] = {g.nx, g.ny, g.nz, g.nw};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int cs[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) cs[a] = wrapi(c[a] + Lat<D>::E[i][a], n[a]);
        const int src = node_index(g, cs);
        const double t = th0[src];
        double eg = 0.0, ax = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int e = Lat<D>::E[i][a];
            if (e == 0) continue;
            const double ga = grad ? grad[(int64_t)a * g.V + src] : fd4<D>(th0, g, cs, a, r.inv12dx);
            eg = e == 1 ? eg + ga : eg - ga;
            if (nnz<D>(i) == 1) ax = e == 1 ? ga : -ga;
        }
        const double w = weight<D>(i, r);
        dst[slot<Q>(i, k)] = w * t - r.dx * w * eg - corr * ax;
    }
}

// ---------------------------------------------------------------------------
// macroscopic output, state conversions
// ---------------------------------------------------------------------------
// theta = sum f, u_a = (2 - s1) c j_a / theta and grad_a theta = -(3 s1/dx) j_a
// with j_a = sum_i e_{ia} f_i (Sec. III.C; sum_i e_i w_i = 0, so j needs no
// equilibrium subtracted).  Any of the three outputs may be NULL.
template <int D>
__global__ void __launch_bounds__(256) k_macro(const double* __restrict__ src,
                                               double* __restrict__ theta, double* __restrict__ u,
                                               double* __restrict__ grad, Geo g, Rates r) {
    constexpr int Q = Lat<D>::Q;
    int c[4];
    if (!thread_node<D>(g, c)) return;
    const Nbr nb = make_nbr<D>(c, g);
    double f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = src[slot<Q>(i, pull_index<D>(nb, i))];
    double th = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) th += f[i];
    const int k = node_index(g, c);
    if (theta) theta[k] = th;
    if (u || grad) {
        const double inv = r.ucoef / th;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double j = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) j = LBM_SADD(j, Lat<D>::E[i][a], f[i]);
            if (u) u[(int64_t)a * g.V + k] = j * inv;
            if (grad) grad[(int64_t)a * g.V + k] = r.gcoef * j;
        }
    }
}

template <int D>
__global__ void __launch_bounds__(256) k_get_state(const double* __restrict__ src,
                                                   double* __restrict__ dense, Geo g) {
    constexpr int Q = Lat<D>::Q;
    int c[4];
    if (!thread_node<D>(g, c)) return;
    const Nbr nb = make_nbr<D>(c, g);
    const int k = node_index(g, c);
#pragma unroll
    for (int i = 0; i < Q; ++i) dense[(int64_t)i * g.V + k] = src[slot<Q>(i, pull_index<D>(nb, i))];
}

template <int D>
__global__ void __launch_bounds__(256) k_set_state(const double* __restrict__ dense,
                                                   double* __restrict__ dst, Geo g) {
    constexpr int Q = Lat<D>::Q;
    int c[4];
    if (!thread_node<D>(g, c)) return;
    const Nbr nb = make_nbr<D>(c, g);
    const int k = node_index(g, c);
#pragma unroll
    for (int i = 0; i < Q; ++i) dst[slot<Q>(i, k)] = dense[(int64_t)i * g.V + push_index<D>(nb, i)];
}

// Canonical (no stream shift) conversions between a dense q x V array and
// the chunked layout, for distribution-shaped adjoint buffers.
template <int D>
__global__ void __launch_bounds__(256) k_layout_from_dense(const double* __restrict__ dense,
                                                           double* __restrict__ buf, Geo g) {
    constexpr int Q = Lat<D>::Q;
    int c[4];
    if (!thread_node<D>(g, c)) return;
    const int k = node_index(g, c);
#pragma unroll
    for (int i = 0; i < Q; ++i) buf[slot<Q>(i, k)] = dense[(int64_t)i * g.V + k];
}

template <int D>
__global__ void __launch_bounds__(256) k_layout_to_dense(const double* __restrict__ buf,
                                                         double* __restrict__ dense, Geo g) {
    constexpr int Q = Lat<D>::Q;
    int c[4];
    if (!thread_node<D>(g, c)) return;
    const int k = node_index(g, c);
#pragma unroll
    for (int i = 0; i < Q; ++i) dense[(int64_t)i * g.V + k] = buf[slot<Q>(i, k)];
}

// Sets *flag when theta = sum_i f_i of some node of the state is not finite
// and positive (a diverged or corrupted run: u = -2 nu grad theta / theta
// needs theta > 0).
template <int D>
__global__ void __launch_bounds__(256) k_check_state(const double* __restrict__ src, int* flag,
                                                     Geo g) {
    constexpr int Q = Lat<D>::Q;
    int c[4];
    if (!thread_node<D>(g, c)) return;
    const Nbr nb = make_nbr<D>(c, g);
    double th = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) th += src[slot<Q>(i, pull_index<D>(nb, i))];
    if (!(th > 0.0) || !isfinite(th)) atomicOr(flag, 1);
}

__global__ void __launch_bounds__(256) k_check_theta(const double* __restrict__ th, int64_t n,
                                                     int* flag) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double v = th[i];
    if (!(v > 0.0) || !isfinite(v)) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) k_macro_adjoint(const double* __restrict__ src,
                                                       const double* __restrict__ gth,
                                                       const double* __restrict__ gu,
                                                       double* __restrict__ lam,
                                                       double* __restrict__ partials, Geo g,
                                                       Rates r) {
    constexpr int Q = Lat<D>::Q;
    int c[4];
    double ge = 0.0;
    if (thread_node<D>(g, c)) {
        const Nbr nb = make_nbr<D>(c, g);
        const int k = node_index(g, c);
        double f[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i] = src[slot<Q>(i, pull_index<D>(nb, i))];
        double th = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) th += f[i];
        const double inv = 1.0 / th;
        const double gt = gth ? gth[k] : 0.0;
        double base = gt, coef[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double j = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) j = LBM_SADD(j, Lat<D>::E[i][a], f[i]);
            const double ga = gu ? gu[(int64_t)a * g.V + k] : 0.0;
            const double ua = r.ucoef * j * inv;
            // d u_a / d f_i = (2 - s1) c e_ia / theta - u_a / theta
            base -= ga * ua * inv;
            coef[a] = ga * r.ucoef * inv;
            // d u_a / d eps = -s1' c j_a / theta
            ge += ga * (-r.ds1) * r.c * j * inv;
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            double v = base;
#pragma unroll
            for (int a = 0; a < D; ++a) v = LBM_SADD(v, Lat<D>::E[i][a], coef[a]);
            lam[slot<Q>(i, k)] = v;
        }
    }
    const double s = block_sum(ge);
    if (threadIdx.x == 0 && threadIdx.y == 0) partials[block_linear()] = s;
}

// lam_out(x) = C^T mu(x), mu_i(x) = lam_in_i(x + e_i); eps part <mu, C' f^n(x)>.
// One partial per block; blocks past the grid up to ntab - 1 are written zero.
// RIN: the state was written by a collision (twins read as in k_step).
template <int D, bool RIN = false>
__global__ void __launch_bounds__(256) k_adjoint_step(const double* __restrict__ state,
                                                      const double* __restrict__ lin,
                                                      double* __restrict__ lout,
                                                      double* __restrict__ partials,
                                                      int64_t ntab, Geo g, Rates r) {
    constexpr int Q = Lat<D>::Q;
    int c[4];
    double ge = 0.0;
    if (thread_node<D>(g, c)) {
        const Nbr nb = make_nbr<D>(c, g);
        const int k = node_index(g, c);
        double f[Q], mu[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            f[i] = state[slot<Q>(RIN ? twin<D>(i) : i, pull_index<D>(nb, i))];
            mu[i] = lin[slot<Q>(i, push_index<D>(nb, i))];
        }
        double df[Q];
        collide_deps<D>(f, r, df);
#pragma unroll
        for (int i = 0; i < Q; ++i) ge += mu[i] * df[i];
        double lam[Q];
        collide_adjoint<D>(mu, r, lam);
#pragma unroll
        for (int i = 0; i < Q; ++i) lout[slot<Q>(i, k)] = lam[i];
    }
    const double s = block_sum(ge);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        const int64_t b = block_linear();
        const int64_t nb = (int64_t)gridDim.x * gridDim.y * gridDim.z;
        partials[b] = s;
        for (int64_t t = nb + b; t < ntab; t += nb) partials[t] = 0.0;
    }
}

// h_a(x) = d L / d g_a(x) for the gradient input of the initialisation:
//   h_a = -dx [ sum_i w_i e_ia lam_i + (1/s1 - 1)(1/6)(lam_{+a} - lam_{-a}) ].
template <int D>
__device__ __forceinline__ double init_h(const double* __restrict__ lam, const Geo& g, int k,
                                         int a, const Rates& r) {
    constexpr int Q = Lat<D>::Q;
    double s = 0.0, ax = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int e = Lat<D>::E[i][a];
        if (e == 0) continue;
        const double l = lam[slot<Q>(i, k)];
        const double wl = weight<D>(i, r) * l;
        s = e == 1 ? s + wl : s - wl;
        if (nnz<D>(i) == 1) ax = e == 1 ? ax + l : ax - l;
    }
    return -r.dx * (s + r.inv_s1_m1 * (1.0 / 6.0) * ax);
}

template <int D>
__global__ void __launch_bounds__(256) k_init_adjoint(const double* __restrict__ th0,
                                                      const double* __restrict__ grad,
                                                      const double* __restrict__ lam,
                                                      double* __restrict__ gth,
                                                      double* __restrict__ ggrad,
                                                      double* __restrict__ partials, Geo g,
                                                      Rates r) {
    constexpr int Q = Lat<D>::Q;
    int c[4];
    double ge = 0.0;
    if (thread_node<D>(g, c)) {
        const int k = node_index(g, c);
        double l[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) l[i] = lam[slot<Q>(i, k)];
        double gt = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) gt += weight<D>(i, r) * l[i];
        double gv[D];
#pragma unroll
        for (int a = 0; a < D; ++a)
            gv[a] = grad ? grad[(int64_t)a * g.V + k] : fd4<D>(th0, g, c, a, r.inv12dx);
        if (grad) {
            if (ggrad) {
#pragma unroll
                for (int a = 0; a < D; ++a) ggrad[(int64_t)a * g.V + k] = init_h<D>(lam, g, k, a, r);
            }
        } else {
            // g_theta0 += sum_a D_a^T h_a, D_a^T h(x) = (-h(x-2) + 8h(x-1) - 8h(x+1) + h(x+2)) / (12 dx)
            const int n[4] = {g.nx, g.ny, g.nz, g.nw};
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int off[4] = {-2, -1, 1, 2};
                const double cf[4] = {-1.0, 8.0, -8.0, 1.0};
                double acc = 0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    int cc[4] = {c[0], c[1], c[2], c[3]};
                    cc[a] = wrapi(c[a] + off[t], n[a]);
                    acc += cf[t] * init_h<D>(lam, g, node_index(g, cc), a, r);
                }
                gt += acc * r.inv12dx;
            }
        }
        gth[k] = gt;
        // d f0_i / d eps = w_i' theta0 - dx w_i' (e_i . g) - (d(1/s1)/deps)(dx/6) (+-g_a on axis i)
        const double t0 = th0[k];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            double eg = 0.0, ax = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int e = Lat<D>::E[i][a];
                if (e == 0) continue;
                eg = e == 1 ? eg + gv[a] : eg - gv[a];
                if (nnz<D>(i) == 1) ax = e == 1 ? gv[a] : -gv[a];
            }
            const double dw = dweight<D>(i, r);
            const double df = dw * t0 - r.dx * dw * eg - r.dinv_s1 * r.dx * (1.0 / 6.0) * ax;
            ge += l[i] * df;
        }
    }
    const double s = block_sum(ge);
    if (threadIdx.x == 0 && threadIdx.y == 0) partials[block_linear()] = s;
}

// *g_eps += sum of the partials; then, if g_nu != NULL, *g_nu = nu_scale * *g_eps
// (dL/dnu = (dt/dx^2) dL/deps, since eps = nu dt/dx^2).
__global__ void __launch_bounds__(256) k_finalize(const double* __restrict__ partials, int64_t n,
                                                  double* g_eps, double* g_nu, double nu_scale) {
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) v += partials[i];
    const double s = block_sum(v);
    if (threadIdx.x == 0) {
        const double ge = *g_eps + s;
        *g_eps = ge;
        if (g_nu) *g_nu = nu_scale * ge;
    }
}

// The reductions of k_finalize for m tables: block j sums table j with the
// same tree into sums[j]; k_accumulate then adds sums[m-1], ..., sums[0] to
// *g_eps one at a time, the order of m k_finalize launches.
__global__ void __launch_bounds__(256) k_table_sums(const double* __restrict__ partials, int64_t n,
                                                    double* __restrict__ sums) {
    const double* p = partials + (int64_t)blockIdx.x * n;
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) v += p[i];
    const double s = block_sum(v);
    if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

__global__ void __launch_bounds__(64) k_accumulate(const double* __restrict__ sums, int64_t m,
                                                   double* g_eps) {
    if (threadIdx.x != 0) return;
    double acc = *g_eps;
    for (int64_t j = m - 1; j >= 0; --j) acc += sums[j];
    *g_eps = acc;
}

// ---------------------------------------------------------------------------
// Burgers front end: theta0 from the initial velocity u0 (inverse Cole-Hopf
// transformation, Sec. II: u = -2 nu grad(theta)/theta, so theta0 =
// exp(-phi/(2 nu)) with grad(phi) = u0).  phi is integrated along the path
// that runs along x_0 at x_1 = .. = 0, then along x_1 at x_2 = .. = 0, and so
// on; each cell integral uses the cubic through four nodes,
//     int_{x_j}^{x_j+1} u = dx (-u_{j-1} + 13 u_j + 13 u_{j+1} - u_{j+2}) / 24,
// (periodic indices).  phi = 0 at the origin.
// ---------------------------------------------------------------------------

// Pass for axis a: one thread per line (c_0..c_{a-1}, *, 0..0); writes the
// running integral along x_a into part_a[c_0 + n_0 (c_1 + ... n_{a-1} c_a)]
// (the index of the node restricted to its first a + 1 coordinates).
__global__ void __launch_bounds__(256) k_potential_axis(const double* __restrict__ u_a,
                                                        double* __restrict__ part, Geo g, int a,
                                                        int64_t nlines, double dx) {
    const int64_t line = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (line >= nlines) return;
    const int n[4] = {g.nx, g.ny, g.nz, g.nw};
    int c[4] = {0, 0, 0, 0};
    int64_t rem = line;
    for (int b = 0; b < a; ++b) {
        c[b] = (int)(rem % n[b]);
        rem /= n[b];
    }
    const int na = n[a];
    int64_t lead = 1;  // stride of axis a in the restricted index
    for (int b = 0; b < a; ++b) lead *= n[b];
    auto u_at = [&](int j) {
        int cc[4] = {c[0], c[1], c[2], c[3]};
        cc[a] = wrapi(j, na);
        return u_a[node_index(g, cc)];
    };
    double phi = 0.0;
    part[line] = 0.0;
    for (int j = 0; j + 1 < na; ++j) {
        phi += dx * ((13.0 * (u_at(j) + u_at(j + 1)) - (u_at(j - 1) + u_at(j + 2))) / 24.0);
        part[line + lead * (j + 1)] = phi;
    }
}

// theta0 = exp(-(sum_a part_a)/(2 nu)); grad theta0 = -u0 theta0/(2 nu).
template <int D>
__global__ void __launch_bounds__(256) k_theta_from_potential(const double* __restrict__ u0,
                                                              const double* __restrict__ parts,
                                                              double* __restrict__ theta,
                                                              double* __restrict__ grad, Geo g,
                                                              double inv2nu) {
    int c[4];
    if (!thread_node<D>(g, c)) return;
    const int n[4] = {g.nx, g.ny, g.nz, g.nw};
    double phi = 0.0;
    int64_t off = 0, restricted = 0, stride = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        restricted += stride * c[a];
        stride *= n[a];
        phi += parts[off + restricted];
        off += stride;
    }
    const int k = node_index(g, c);
    const double th = exp(-phi * inv2nu);
    theta[k] = th;
    if (grad) {
#pragma unroll
        for (int a = 0; a < D; ++a) grad[(int64_t)a * g.V + k] = -u0[(int64_t)a * g.V + k] * th * inv2nu;
    }
}

// ---------------------------------------------------------------------------
// batched 2-D step over a tile table
// ---------------------------------------------------------------------------
// One block per tile.  tx > 0: a tx x (256/tx) rectangle of one instance at
// (x0, y0); tx == 0: 256 consecutive node indices of one instance starting at
// x0, crossing row ends, so no lane idles except at the instance's last tile.
template <bool RIN, bool WOUT>
__global__ void __launch_bounds__(256) k_batch_step(const BatchInst* __restrict__ insts,
                                                    const BatchTile* __restrict__ tiles, int tx,
                                                    int log2tx, const double* __restrict__ src,
                                                    double* __restrict__ dst) {
    constexpr int Q = 9;
    const BatchTile t = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const BatchInst& in = insts[t.inst];
    const int tid = threadIdx.x;
    int x, y;
    if (tx == 0) {
        const int k = t.x0 + tid;
        if (k >= in.nx * in.ny) return;
        y = k / in.nx;
        x = k - y * in.nx;
    } else {
        x = t.x0 + (tid & (tx - 1));
        y = t.y0 + (tid >> log2tx);
        if (x >= in.nx || y >= in.ny) return;
    }
    Geo g;
    g.nx = in.nx;
    g.ny = in.ny;
    g.nz = 1;
    g.nw = 1;
    g.V = (int64_t)in.nx * in.ny;
    const int c[4] = {x, y, 0, 0};
    const Nbr nb = make_nbr<2>(c, g);
    const double* s = src + in.offset;
    double* d = dst + in.offset;
    double f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = s[slot<Q>(RIN ? twin<2>(i) : i, pull_index<2>(nb, i))];
    const Rates r = in.r;
    collide<2>(f, r);
    const int k = y * g.nx + x;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        if (!WOUT || twin<2>(i) == i) __builtin_nontemporal_store(f[i], d + slot<Q>(i, k));
}

// ---------------------------------------------------------------------------
// S D2Q9 time steps per pass, two-wave variant for the batched form.
//
// A block of LW_THREADS = 128 threads owns a strip of 128 - 2S columns (112
// at S = 8 against 48 for one wave), which wastes fewer columns on the
// halo and on the ragged last strip of instances 64..1024 nodes wide.  Thread
// t owns column x0 - S + t in every stage; the populations with e_x != 0
// cross between the two waves through LDS, written already shifted by e_x
// (producer column t -> slot t + e_x) so that every consumer reads its own
// column, with a barrier per stage; stages alternate between two LDS buffers
// of 6 x 128 doubles.  Rows are delayed in registers as in the one-wave
// routine.  Same arithmetic, so also bitwise S single steps.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int lw_ex(int i) { return Lat<2>::E[i][0]; }
__host__ __device__ constexpr int lw_ey(int i) { return Lat<2>::E[i][1]; }
// index of population i among those with e_x != 0
__host__ __device__ constexpr int lw_xslot(int i) {
    int s = 0;
    for (int j = 0; j < i; ++j) s += lw_ex(j) != 0;
    return s;
}
// index of population i among those with the same e_y
__host__ __device__ constexpr int lw_yslot(int i) {
    int s = 0;
    for (int j = 0; j < i; ++j) s += lw_ey(j) == lw_ey(i);
    return s;
}

template <int S>
struct LwState {
    double pre[9];      // next input row (prefetched)
    double z[S][3];     // e_y = 0 populations of the previous row, per stage input
    double u[2][S][3];  // e_y = +1 populations of the rows of each parity
};

// One iteration k of the march; P = k & 1.
template <int S, int P, bool OFF32, bool RIN, bool WOUT>
__device__ __forceinline__ void lw_row(LwState<S>& st, double (&lds)[2][6][LW_THREADS], int k,
                                       int kend, const double* __restrict__ src,
                                       double* __restrict__ dst, int nx, int ny, int gx, int ys,
                                       int x0, const FoldedRates& r) {
    constexpr int W = LW_THREADS - 2 * S;
    const int tid = threadIdx.x;
    double f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = st.pre[RIN ? twin<2>(i) : i];
    // (an unconditional prefetch as in ms_row raised this kernel to 260
    // VGPRs, one wave per SIMD, and cost 20 % on the batch)
    if (k < kend) {
        const MsAddr<OFF32> a(wrapi(ys - S + k + 1, ny) * nx + gx);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            if (!RIN || twin<2>(i) == i) st.pre[i] = a.load(src, i);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i)
        if (lw_ex(i) != 0) {
            const int c = tid + lw_ex(i);
            if (c >= 0 && c < LW_THREADS) lds[0][lw_xslot(i)][c] = f[i];
        }
    __syncthreads();
#pragma unroll
    for (int j = 1; j <= S; ++j) {
        // inputs of stage j: stage j-1 rows of iterations k (e_y = -1), k-1
        // (e_y = 0) and k-2 (e_y = +1)
        double in[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double v = lw_ex(i) != 0 ? lds[(j - 1) & 1][lw_xslot(i)][tid] : f[i];
            if (lw_ey(i) == -1) {
                in[i] = v;
            } else if (lw_ey(i) == 0) {
                in[i] = st.z[j - 1][lw_yslot(i)];
                st.z[j - 1][lw_yslot(i)] = v;
            } else {
                in[i] = st.u[P][j - 1][lw_yslot(i)];
                st.u[P][j - 1][lw_yslot(i)] = v;
            }
        }
        // stage j holds valid rows from iteration 2j on, in columns j .. T-1-j
        if (k >= 2 * j && tid >= j && tid < LW_THREADS - j) {
            collide_d2q9(in, r);
            if (j < S) {
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    f[i] = in[i];
                    if (lw_ex(i) != 0) {
                        const int c = tid + lw_ex(i);
                        if (c >= 0 && c < LW_THREADS) lds[j & 1][lw_xslot(i)][c] = in[i];
                    }
                }
            } else if (tid >= S && tid < S + W && x0 - S + tid < nx) {
                const MsAddr<OFF32> a(wrapi(ys - 2 * S + k, ny) * nx + x0 - S + tid);
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    if (!WOUT || twin<2>(i) == i) a.store(dst, i, in[i]);
            }
        }
        if (j < S) __syncthreads();
    }
    // with S odd the last stage reads buffer 0, which the next load rewrites
    if (S & 1) __syncthreads();
}

// Advance rows [ys, ye) of the columns [x0, x0 + LW_THREADS - 2S) of one
// D2Q9 grid by S steps (reads rows ys-S .. ye-1+S and columns x0-S ..
// x0+LW_THREADS-S-1, wrapped periodically).
template <int S, bool OFF32, bool RIN, bool WOUT>
__device__ __forceinline__ void lw_tile(const double* __restrict__ src, double* __restrict__ dst,
                                        int nx, int ny, const FoldedRates& r, int x0, int ys, int ye,
                                        double (&lds)[2][6][LW_THREADS]) {
    const int gx = wrapi(x0 - S + (int)threadIdx.x, nx);
    const int kend = ye - ys + 2 * S - 1;
    LwState<S> st;
    {
        const MsAddr<OFF32> a(wrapi(ys - S, ny) * nx + gx);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            if (!RIN || twin<2>(i) == i) st.pre[i] = a.load(src, i);
    }
#pragma unroll
    for (int j = 0; j < S; ++j)
#pragma unroll
        for (int a = 0; a < 3; ++a) st.z[j][a] = st.u[0][j][a] = st.u[1][j][a] = 0.0;
    // row pairs in the loop, a last odd row after it (as in ms_tile)
    int k = 0;
    for (; k + 1 <= kend; k += 2) {
        lw_row<S, 0, OFF32, RIN, WOUT>(st, lds, k, kend, src, dst, nx, ny, gx, ys, x0, r);
        lw_row<S, 1, OFF32, RIN, WOUT>(st, lds, k + 1, kend, src, dst, nx, ny, gx, ys, x0, r);
    }
    if (k <= kend) lw_row<S, 0, OFF32, RIN, WOUT>(st, lds, k, kend, src, dst, nx, ny, gx, ys, x0, r);
}


// Batched S-step pass: tile (inst, x0, y0, y1) = rows [y0, y1) of the strip
// at x0 (batch_strip_width(S) columns) of one instance.  OFF32: every
// instance's state is under 4 GiB (MsAddr<true> from the instance's start).
// RIN / WOUT as for k_step.
template <int S, bool OFF32, bool RIN, bool WOUT>
__global__ void __launch_bounds__(LW_THREADS) k_batch_steps(const BatchInst* __restrict__ insts,
                                                            const BatchTile* __restrict__ tiles,
                                                            const double* __restrict__ src,
                                                            double* __restrict__ dst) {
    __shared__ double lds[2][6][LW_THREADS];
    const BatchTile t = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const BatchInst& in = insts[t.inst];
    lw_tile<S, OFF32, RIN, WOUT>(src + in.offset, dst + in.offset, in.nx, in.ny, folded(in.r),
                                 t.x0, t.y0, t.pad, lds);
}

// The same pass with the one-wave march of k_steps_d2q9: tile (inst, x0,
// y0, y1) = rows [y0, y1) of the strip at x0 (strip_width(S) columns).
template <int S, bool OFF32, bool RIN, bool WOUT>
__global__ void __launch_bounds__(MS_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
k_batch_steps_w(const BatchInst* __restrict__ insts, const BatchTile* __restrict__ tiles,
                const double* __restrict__ src, double* __restrict__ dst) {
    const BatchTile t = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const BatchInst& in = insts[t.inst];
    ms_tile<S, false, OFF32, true, RIN, WOUT>(src + in.offset, dst + in.offset, in.nx, in.ny,
                                              folded(in.r), t.x0, t.y0, t.pad, 0);
}

template <typename F>
hipError_t dispatch(int d, F&& f) {
    switch (d) {
        case 1: return f(std::integral_constant<int, 1>{});
        case 2: return f(std::integral_constant<int, 2>{});
        case 3: return f(std::integral_constant<int, 3>{});
        case 4: return f(std::integral_constant<int, 4>{});
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

Launch launch_shape(int d, const Geo& g) {
    Launch L;
    if (d == 1) {
        L.block = dim3(B1, 1, 1);
        L.grid = dim3((unsigned)((g.nx + B1 - 1) / B1), 1, 1);
    } else {
        // 256 threads: a whole row segment of 256 nodes, or for rows of at
        // most 128 (64) nodes 2 (4) rows of 128 (64), so that short rows do
        // not leave most of a block idle (64^4: one row of 64 per block left
        // three of its four waves without a node)
        const int bx = g.nx > 128 ? BX : (g.nx > 64 ? 128 : 64);
        const int by = BX * BY / bx;
        L.block = dim3(bx, by, 1);
        L.grid = dim3((unsigned)((g.nx + bx - 1) / bx), (unsigned)((g.ny + by - 1) / by),
                      (unsigned)(d >= 3 ? g.nz * g.nw : 1));
    }
    L.nblocks = (int64_t)L.grid.x * L.grid.y * L.grid.z;
    return L;
}

#define LBM_LAUNCH(kern, ...)                                                     \
    dispatch(d, [&](auto dc) {                                                    \
        constexpr int DD = decltype(dc)::value;                                   \
        const Launch L = launch_shape(DD, g);                                     \
        hipLaunchKernelGGL(kern<DD>, L.grid, L.block, 0, st, __VA_ARGS__);        \
        return hipGetLastError();                                                 \
    })

// (rin, wout) as template arguments of a kernel.
template <typename F>
hipError_t dispatch_io(bool rin, bool wout, F&& f) {
    if (rin)
        return wout ? f(std::true_type{}, std::true_type{}) : f(std::true_type{}, std::false_type{});
    return wout ? f(std::false_type{}, std::true_type{}) : f(std::false_type{}, std::false_type{});
}

hipError_t launch_step(int d, const Geo& g, const Rates& r, const double* src, double* dst,
                       hipStream_t st, bool rin, bool wout) {
    return dispatch(d, [&](auto dc) {
        constexpr int DD = decltype(dc)::value;
        const Launch L = launch_shape(DD, g);
        if constexpr (DD == 1) {  // D1Q3 has no twins
            hipLaunchKernelGGL((k_step<1>), L.grid, L.block, 0, st, src, dst, g, r);
            return hipGetLastError();
        } else {
            return dispatch_io(rin, wout, [&](auto ri, auto wo) {
                hipLaunchKernelGGL((k_step<DD, decltype(ri)::value, decltype(wo)::value>), L.grid,
                                   L.block, 0, st, src, dst, g, r);
                return hipGetLastError();
            });
        }
    });
}

hipError_t launch_step_resident1(const Geo& g, const Rates& r, const double* src, double* dst,
                                int64_t nsteps, const double* walls, double* wall_now,
                                hipStream_t st) {
    if (g.nx > RESIDENT_MAX_1D || g.ny != 1 || g.nz != 1 || g.nw != 1) return hipErrorInvalidValue;
    if (walls && (!wall_now || g.nx < 2)) return hipErrorInvalidValue;
    const int n = g.nx;
#define LBM_WAVE1(PER, PERIODIC)                                                                  \
    hipLaunchKernelGGL((k_step_wave1<PER, PERIODIC>), dim3(1), dim3(64), 0, st, src, dst, n, nsteps, \
                       r, walls, wall_now)
    if (!walls) {
        // periodic grids of exactly 64, 128 or 256 nodes: one wave, lane rotations
        if (n == 64) { LBM_WAVE1(1, true); return hipGetLastError(); }
        if (n == 128) { LBM_WAVE1(2, true); return hipGetLastError(); }
        if (n == 256) { LBM_WAVE1(4, true); return hipGetLastError(); }
    } else {
        if (n <= 64) { LBM_WAVE1(1, false); return hipGetLastError(); }
        if (n <= 128) { LBM_WAVE1(2, false); return hipGetLastError(); }
        if (n <= 256) { LBM_WAVE1(4, false); return hipGetLastError(); }
    }
#undef LBM_WAVE1
#define LBM_RES1(T, PER)                                                                          \
    hipLaunchKernelGGL((k_step_resident1<T, PER>), dim3(1), dim3(T), 0, st, src, dst, n, nsteps, r, \
                       walls, wall_now)
    if (n <= 64) LBM_RES1(64, 1);
    else if (n <= 128) LBM_RES1(64, 2);
    else if (n <= 256) LBM_RES1(128, 2);
    else if (n <= 512) LBM_RES1(256, 2);
    else if (n <= 1024) LBM_RES1(256, 4);
    else LBM_RES1(256, 8);
#undef LBM_RES1
    static_assert(256 * 8 >= RESIDENT_MAX_1D, "resident shapes cover RESIDENT_MAX_1D");
    return hipGetLastError();
}

static dim3 grid_1d(int n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_step_wall1(const Geo& g, const Rates& r, const double* src, double* dst,
                             const double* wall, hipStream_t st) {
    if (g.nx < 2 || g.ny != 1 || g.nz != 1 || g.nw != 1 || !wall) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_step_wall1, grid_1d(g.nx), dim3(256), 0, st, src, dst, g.nx, r, wall);
    return hipGetLastError();
}

hipError_t launch_macro_wall1(const Geo& g, const Rates& r, const double* state, double* theta,
                              double* u, double* grad, const double* wall, hipStream_t st) {
    if (g.nx < 2 || g.ny != 1 || g.nz != 1 || g.nw != 1 || !wall) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_macro_wall1, grid_1d(g.nx), dim3(256), 0, st, state, theta, u, grad, g.nx,
                       r, wall);
    return hipGetLastError();
}

hipError_t launch_get_state_wall1(const Geo& g, const double* state, double* dense,
                                  const double* wall, hipStream_t st) {
    if (g.nx < 2 || g.ny != 1 || g.nz != 1 || g.nw != 1 || !wall) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_get_state_wall1, grid_1d(g.nx), dim3(256), 0, st, state, dense, g.nx, wall);
    return hipGetLastError();
}

hipError_t launch_wall_from_dense1(const Geo& g, const double* dense, double* wall,
                                   hipStream_t st) {
    if (g.nx < 2 || !wall) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_wall_from_dense1, dim3(1), dim3(64), 0, st, dense, g.nx, wall);
    return hipGetLastError();
}

// Rows per segment of an S-step launch.  A one-wave block of k_steps_d2q9
// holds about 240 VGPRs, so a CU runs 8 of them at once: the segments are
// cut so that all blocks fit in one round of 8 x (number of CUs) (fewer,
// longer segments amortise the 2S-row pipeline fill; a partial second round
// costs far more), at least 8 rows, and in more rounds when a segment would
// exceed 512 rows.  Measured minimum (MLUPS at 8 steps per pass): 512^2
// 47,500 at 24 rows, 70,200 at 8; 1024^2 132,000 and 148,300; 2048^2 and
// 4096^2 unchanged (their segments are longer).
// Blocks of k_steps_d2q9 one round holds on the current device (8 per CU),
// looked up once per device.
static int round_slots() {
    constexpr int kMaxDevices = 64;
    static std::atomic<int> cached[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) dev = 0;
    const int d = dev < kMaxDevices ? dev : kMaxDevices - 1;
    int slots = cached[d].load(std::memory_order_relaxed);
    if (slots == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        slots = 8 * cus;
        cached[d].store(slots, std::memory_order_relaxed);
    }
    return slots;
}

// Minimum rows per segment: plain passes 8; the passes of an adjoint
// checkpoint segment (recomputation and reverse sweep) 3, since at the sizes
// the adjoint runs (512^2) they are short of waves (measured per step of a
// 45-step segment at 512^2: 15.1 us at 8 rows, 12.9 us at 3).
constexpr int kMinRows = 8;
constexpr int kMinRowsSegment = 3;

static int steps_rows(const Geo& g, int nstrips, int min_rows) {
    const int slots = round_slots();
    int64_t per_round = slots / nstrips;
    if (per_round < 1) per_round = 1;
    int64_t nseg = per_round;
    int64_t ly = (g.ny + nseg - 1) / nseg;
    while (ly > 512) {
        nseg += per_round;
        ly = (g.ny + nseg - 1) / nseg;
    }
    if (ly < min_rows) ly = min_rows;
    if (ly > g.ny) ly = g.ny;
    return (int)ly;
}

template <int S>
static hipError_t launch_steps_t(const Geo& g, const Rates& r, const double* src, double* dst,
                                 hipStream_t st, bool rin, bool wout) {
    const int w = strip_width(S);
    const int nstrips = (g.nx + w - 1) / w;
    const int ly = steps_rows(g, nstrips, kMinRows);
    const int nseg = (g.ny + ly - 1) / ly;
    const dim3 grid((unsigned)((int64_t)nstrips * nseg));
    return dispatch_io(rin, wout, [&](auto ri, auto wo) {
        constexpr bool RI = decltype(ri)::value, WO = decltype(wo)::value;
        if (d2q9_cached_stores(g))  // both states fit in 256 MB, so under 4 GiB
            hipLaunchKernelGGL((k_steps_d2q9_cached<S, true, RI, WO>), grid, dim3(MS_THREADS), 0,
                               st, src, dst, g, r, ly, nstrips);
        else if (ms_off32(g))
            hipLaunchKernelGGL((k_steps_d2q9<S, true, RI, WO>), grid, dim3(MS_THREADS), 0, st, src,
                               dst, g, r, ly, nstrips);
        else
            hipLaunchKernelGGL((k_steps_d2q9<S, false, RI, WO>), grid, dim3(MS_THREADS), 0, st,
                               src, dst, g, r, ly, nstrips);
        return hipGetLastError();
    });
}

// Planes per segment of a D3Q19 pass: 64, fewer (at least 16) when the grid
// would otherwise give under about 1280 blocks, then evened out over the
// segments.
template <int S>
static hipError_t launch_steps3_t(const Geo& g, const Rates& r, const double* src, double* dst,
                                  hipStream_t st, bool rin, bool wout) {
    const int ntx = (g.nx + tile_width3(S) - 1) / tile_width3(S);
    const int nty = (g.ny + tile_height3(S) - 1) / tile_height3(S);
    int64_t lz = ((int64_t)g.nz * ntx * nty + 1279) / 1280;
    if (lz > 64) lz = 64;
    if (lz < 16) lz = 16;
    if (lz > g.nz) lz = g.nz;
    // segments of equal length: a short last segment is mostly pipeline fill
    // (512 x 512 x 64: 58 + 6 planes gave 16.6 GLUPS, 32 + 32 planes 25.6)
    lz = (g.nz + (g.nz + lz - 1) / lz - 1) / ((g.nz + lz - 1) / lz);
    const int64_t nseg = (g.nz + lz - 1) / lz;  // every segment non-empty
    const int64_t nb = (int64_t)ntx * nty * nseg;
    if (nb > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
    // buffer loads need the chunks of one z-plane under 2 GiB (planes up to
    // about 14 M nodes)
    const int64_t plane = (int64_t)g.nx * g.ny;
    const bool buf = (plane / 4096 + 2) * 19 * 4096 * 8 < ((int64_t)1 << 31);
    return dispatch_io(rin, wout, [&](auto ri, auto wo) {
        constexpr bool RI = decltype(ri)::value, WO = decltype(wo)::value;
        if (RI && buf)
            hipLaunchKernelGGL((k_steps_d3q19<S, RI, WO, RI>), dim3((unsigned)nb),
                               dim3(M3_THREADS), 0, st, src, dst, g, r, (int)lz, ntx, nty);
        else
            hipLaunchKernelGGL((k_steps_d3q19<S, RI, WO, false>), dim3((unsigned)nb),
                               dim3(M3_THREADS), 0, st, src, dst, g, r, (int)lz, ntx, nty);
        return hipGetLastError();
    });
}

hipError_t launch_steps3(int nsteps, const Geo& g, const Rates& r, const double* src, double* dst,
                         hipStream_t st, bool rin, bool wout) {
    if (g.nw != 1) return hipErrorInvalidValue;
    switch (nsteps) {
        case 2: return launch_steps3_t<2>(g, r, src, dst, st, rin, wout);
        default: return hipErrorInvalidValue;
    }
}

template <int S>
static hipError_t launch_steps_all_t(const Geo& g, const Rates& r, const double* src, double* out,
                                     int64_t stride, hipStream_t st, bool rin, bool wout) {
    const int w = strip_width(S);
    const int nstrips = (g.nx + w - 1) / w;
    const int ly = steps_rows(g, nstrips, kMinRowsSegment);
    const dim3 grid((unsigned)((int64_t)nstrips * ((g.ny + ly - 1) / ly)));
    const bool off32 = ms_off32(g);
    return dispatch_io(rin, wout, [&](auto ri, auto wo) {
        constexpr bool RI = decltype(ri)::value, WO = decltype(wo)::value;
        if (off32)
            hipLaunchKernelGGL((k_steps_d2q9_all<S, true, RI, WO>), grid, dim3(MS_THREADS), 0, st,
                               src, out, stride, g, r, ly, nstrips);
        else
            hipLaunchKernelGGL((k_steps_d2q9_all<S, false, RI, WO>), grid, dim3(MS_THREADS), 0, st,
                               src, out, stride, g, r, ly, nstrips);
        return hipGetLastError();
    });
}

hipError_t launch_steps_all(int nsteps, const Geo& g, const Rates& r, const double* src,
                            double* out, int64_t stride, hipStream_t st, bool rin, bool wout) {
    switch (nsteps) {
        case 2: return launch_steps_all_t<2>(g, r, src, out, stride, st, rin, wout);
        case 4: return launch_steps_all_t<4>(g, r, src, out, stride, st, rin, wout);
        case 8: return launch_steps_all_t<8>(g, r, src, out, stride, st, rin, wout);
        default: return hipErrorInvalidValue;
    }
}

template <int S>
static int64_t adjoint_steps_blocks_t(const Geo& g) {
    const int w = strip_width(S);
    const int64_t nstrips = (g.nx + w - 1) / w;
    const int ly = steps_rows(g, (int)nstrips, kMinRowsSegment);
    return nstrips * ((g.ny + ly - 1) / ly);
}

int64_t adjoint_steps_table(const Geo& g) {
    return std::max(adjoint_steps_blocks_t<2>(g), adjoint_steps_blocks_t<4>(g));
}

template <int S>
static hipError_t launch_adjoint_steps_t(const Geo& g, const Rates& r, const double* lam_in,
                                         double* lam_out, const double* ftop, int64_t stride,
                                         double* partials, int64_t ntab, hipStream_t st,
                                         bool rin) {
    const int w = strip_width(S);
    const int nstrips = (g.nx + w - 1) / w;
    const int ly = steps_rows(g, nstrips, kMinRowsSegment);
    const int64_t nb = (int64_t)nstrips * ((g.ny + ly - 1) / ly);
    if (nb > ntab || ntab > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    if (rin)
        hipLaunchKernelGGL((k_adjoint_steps_d2q9<S, true>), dim3((unsigned)nb), dim3(MS_THREADS),
                           0, st, lam_in, lam_out, ftop, stride, partials, (int)ntab, g, r, ly,
                           nstrips);
    else
        hipLaunchKernelGGL((k_adjoint_steps_d2q9<S, false>), dim3((unsigned)nb), dim3(MS_THREADS),
                           0, st, lam_in, lam_out, ftop, stride, partials, (int)ntab, g, r, ly,
                           nstrips);
    return hipGetLastError();
}

hipError_t launch_adjoint_steps(int nsteps, const Geo& g, const Rates& r, const double* lam_in,
                                double* lam_out, const double* ftop, int64_t stride,
                                double* partials, int64_t ntab, hipStream_t st, bool rin) {
    switch (nsteps) {
        case 2:
            return launch_adjoint_steps_t<2>(g, r, lam_in, lam_out, ftop, stride, partials, ntab,
                                             st, rin);
        case 4:
            return launch_adjoint_steps_t<4>(g, r, lam_in, lam_out, ftop, stride, partials, ntab,
                                             st, rin);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_steps(int nsteps, const Geo& g, const Rates& r, const double* src, double* dst,
                        hipStream_t st, bool rin, bool wout) {
    switch (nsteps) {
        case 2: return launch_steps_t<2>(g, r, src, dst, st, rin, wout);
        case 4: return launch_steps_t<4>(g, r, src, dst, st, rin, wout);
        case 8: return launch_steps_t<8>(g, r, src, dst, st, rin, wout);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_init(int d, const Geo& g, const Rates& r, const double* theta0,
                       const double* grad, double* dst, hipStream_t st) {
    return LBM_LAUNCH(k_init, theta0, grad, dst, g, r);
}

hipError_t launch_macro(int d, const Geo& g, const Rates& r, const double* state, double* theta,
                        double* u, double* grad, hipStream_t st) {
    return LBM_LAUNCH(k_macro, state, theta, u, grad, g, r);
}

hipError_t launch_check_state(int d, const Geo& g, const double* state, int* flag,
                              hipStream_t st) {
    return LBM_LAUNCH(k_check_state, state, flag, g);
}

hipError_t launch_get_state(int d, const Geo& g, const double* state, double* dense,
                            hipStream_t st) {
    return LBM_LAUNCH(k_get_state, state, dense, g);
}

hipError_t launch_set_state(int d, const Geo& g, const double* dense, double* state,
                            hipStream_t st) {
    return LBM_LAUNCH(k_set_state, dense, state, g);
}

hipError_t launch_layout_from_dense(int d, const Geo& g, const double* dense, double* buf,
                                   hipStream_t st) {
    return LBM_LAUNCH(k_layout_from_dense, dense, buf, g);
}

hipError_t launch_layout_to_dense(int d, const Geo& g, const double* buf, double* dense,
                                 hipStream_t st) {
    return LBM_LAUNCH(k_layout_to_dense, buf, dense, g);
}

int64_t potential_workspace(int d, const Geo& g) {
    const int n[4] = {g.nx, g.ny, g.nz, g.nw};
    int64_t total = 0, prod = 1;
    for (int a = 0; a < d; ++a) {
        prod *= n[a];
        total += prod;
    }
    return total;
}

hipError_t launch_theta_from_velocity(int d, const Geo& g, double dx, double nu, const double* u0,
                                      double* work, double* theta, double* grad,
                                      hipStream_t st) {
    const int n[4] = {g.nx, g.ny, g.nz, g.nw};
    int64_t off = 0, nlines = 1;
    for (int a = 0; a < d; ++a) {
        hipLaunchKernelGGL(k_potential_axis, dim3((unsigned)((nlines + 255) / 256)), dim3(256), 0,
                           st, u0 + (int64_t)a * g.V, work + off, g, a, nlines, dx);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        nlines *= n[a];
        off += nlines;
    }
    const double inv2nu = 1.0 / (2.0 * nu);
    return LBM_LAUNCH(k_theta_from_potential, u0, work, theta, grad, g, inv2nu);
}

hipError_t launch_check_theta(const double* theta, int64_t n, int* flag, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_theta, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, theta,
                       n, flag);
    return hipGetLastError();
}

hipError_t launch_macro_adjoint(int d, const Geo& g, const Rates& r, const double* state,
                                const double* g_theta, const double* g_u, double* lambda,
                                double* partials, hipStream_t st) {
    return LBM_LAUNCH(k_macro_adjoint, state, g_theta, g_u, lambda, partials, g, r);
}

hipError_t launch_adjoint_step(int d, const Geo& g, const Rates& r, const double* state,
                               const double* lam_in, double* lam_out, double* partials,
                               int64_t ntab, hipStream_t st, bool rin) {
    if (ntab < launch_shape(d, g).nblocks) return hipErrorInvalidValue;
    return dispatch(d, [&](auto dc) {
        constexpr int DD = decltype(dc)::value;
        const Launch L = launch_shape(DD, g);
        constexpr bool HAS_TWINS = DD > 1;  // D1Q3 has none
        if (HAS_TWINS && rin)
            hipLaunchKernelGGL((k_adjoint_step<DD, HAS_TWINS>), L.grid, L.block, 0, st, state,
                               lam_in, lam_out, partials, ntab, g, r);
        else
            hipLaunchKernelGGL((k_adjoint_step<DD, false>), L.grid, L.block, 0, st, state, lam_in,
                               lam_out, partials, ntab, g, r);
        return hipGetLastError();
    });
}

hipError_t launch_init_adjoint(int d, const Geo& g, const Rates& r, const double* theta0,
                               const double* grad, const double* lambda0, double* g_theta0,
                               double* g_grad, double* partials, hipStream_t st) {
    return LBM_LAUNCH(k_init_adjoint, theta0, grad, lambda0, g_theta0, g_grad, partials, g, r);
}

hipError_t launch_finalize(const double* partials, int64_t n, double* g_eps, hipStream_t st,
                           double* g_nu, double nu_scale) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, partials, n, g_eps, g_nu, nu_scale);
    return hipGetLastError();
}

hipError_t launch_finalize_tables(const double* partials, int64_t n, int64_t m, double* sums,
                                  double* g_eps, hipStream_t st) {
    if (m < 1 || m > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_table_sums, dim3((unsigned)m), dim3(256), 0, st, partials, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_accumulate, dim3(1), dim3(64), 0, st, sums, m, g_eps);
    return hipGetLastError();
}

template <bool OFF32, bool RIN, bool WOUT>
static hipError_t launch_batch_steps_t(int nsteps, const BatchInst* insts, const BatchTile* tiles,
                                       int64_t ntiles, const double* src, double* dst,
                                       bool one_wave, hipStream_t st) {
    const dim3 grid((unsigned)ntiles), block(one_wave ? MS_THREADS : LW_THREADS);
    switch (nsteps * (one_wave ? -1 : 1)) {
#define LBM_BATCH_CASE(S)                                                                      \
    case S: hipLaunchKernelGGL((k_batch_steps<S, OFF32, RIN, WOUT>), grid, block, 0, st, insts, \
                               tiles, src, dst); break;                                        \
    case -S: hipLaunchKernelGGL((k_batch_steps_w<S, OFF32, RIN, WOUT>), grid, block, 0, st,    \
                                insts, tiles, src, dst); break;
        LBM_BATCH_CASE(2)
        LBM_BATCH_CASE(4)
        LBM_BATCH_CASE(8)
#undef LBM_BATCH_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_steps(int nsteps, const BatchInst* insts, const BatchTile* tiles,
                              int64_t ntiles, const double* src, double* dst, bool off32,
                              bool one_wave, hipStream_t st, bool rin, bool wout) {
    if (ntiles <= 0) return hipSuccess;
    return dispatch_io(rin, wout, [&](auto ri, auto wo) {
        constexpr bool RI = decltype(ri)::value, WO = decltype(wo)::value;
        return off32 ? launch_batch_steps_t<true, RI, WO>(nsteps, insts, tiles, ntiles, src, dst,
                                                          one_wave, st)
                     : launch_batch_steps_t<false, RI, WO>(nsteps, insts, tiles, ntiles, src, dst,
                                                           one_wave, st);
    });
}

hipError_t launch_batch_step(const BatchInst* insts, const BatchTile* tiles, int64_t ntiles,
                             int tx, int ty, const double* src, double* dst, hipStream_t st,
                             bool rin, bool wout) {
    (void)ty;
    int log2tx = 0;
    while (tx > 0 && (1 << log2tx) < tx) ++log2tx;
    if (ntiles <= 0) return hipSuccess;
    return dispatch_io(rin, wout, [&](auto ri, auto wo) {
        hipLaunchKernelGGL((k_batch_step<decltype(ri)::value, decltype(wo)::value>),
                           dim3((unsigned)ntiles), dim3(256), 0, st, insts, tiles, tx, log2tx, src,
                           dst);
        return hipGetLastError();
    });
}

}  // namespace lbm
