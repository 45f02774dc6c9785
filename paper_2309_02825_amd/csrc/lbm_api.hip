// C ABI of the solver (declared in include/lbm.h): validation, parameters of
// Theorem 2 (Sec. III.D), buffer bookkeeping and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "lbm.h"
#include "lbm_kernels.h"

using lbm::BatchInst;
using lbm::BatchTile;
using lbm::Geo;
using lbm::Launch;
using lbm::Rates;

namespace {

thread_local std::string g_err;

lb_status fail(lb_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

lb_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return LB_ERR_HIP;
}

#define LB_HIP(call, what)                          \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// Relaxation rates and weights of Theorem 2 (Sec. III.D, parameter solution):
//   s1 = 2/(6 eps + 1), s21 = 24 eps/(6 eps + 1)^2, s22 = 4/(6 eps + 3),
//   w1 = 1/6 - (d-1) eps/3 (1/6 in 1-D), w_{1+2d} = eps/6 (absent in 1-D),
//   w0 = 1 - 2 d w1 - 2 d (d-1) w_{1+2d}  (weight structure, Sec. III.A),
// plus their eps-derivatives for the adjoint.
Rates make_rates(int d, double dx, double dt, double nu) {
    Rates r;
    const double eps = nu * dt / (dx * dx);
    const double a6 = 6.0 * eps + 1.0;
    r.eps = eps;
    r.s1 = 2.0 / a6;
    r.s21 = 24.0 * eps / (a6 * a6);
    r.s22 = 4.0 / (6.0 * eps + 3.0);
    double dw1, dwd;
    if (d == 1) {
        r.w1 = 1.0 / 6.0;
        r.wd = 0.0;
        dw1 = 0.0;
        dwd = 0.0;
    } else {
        r.w1 = 1.0 / 6.0 - (d - 1) * eps / 3.0;
        r.wd = eps / 6.0;
        dw1 = -(d - 1) / 3.0;
        dwd = 1.0 / 6.0;
    }
    r.w0 = 1.0 - 2.0 * d * r.w1 - 2.0 * d * (d - 1) * r.wd;
    r.one_m_s1 = 1.0 - r.s1;
    r.one_m_s21 = 1.0 - r.s21;
    r.one_m_s22 = 1.0 - r.s22;
    r.R4wd = 4.0 * r.wd;
    r.c = dx / dt;
    r.ucoef = (2.0 - r.s1) * r.c;
    // grad theta = -(s1/(dt c_s^2)) sum_i c_i f^ne_i (Sec. III.C) with c_i = c e_i
    // and c_s^2 = c^2/3 on every lattice here
    r.gcoef = -3.0 * r.s1 / dx;
    r.dx = dx;
    r.inv_s1_m1 = 1.0 / r.s1 - 1.0;
    r.inv12dx = 1.0 / (12.0 * dx);
    r.ds1 = -12.0 / (a6 * a6);
    r.ds21 = 24.0 * (1.0 - 6.0 * eps) / (a6 * a6 * a6);
    r.ds22 = -24.0 / ((6.0 * eps + 3.0) * (6.0 * eps + 3.0));
    r.dw1 = dw1;
    r.dwd = dwd;
    r.dw0 = -2.0 * d * dw1 - 2.0 * d * (d - 1) * dwd;
    r.dinv_s1 = 3.0;
    r.f_cj = 0.5 * (1.0 - r.s1);
    r.f_cp = 0.5 * (1.0 - r.s21);
    r.f_ct = r.s21 / 6.0 - 2.0 * (d - 1) * r.wd;
    r.f_cq = 0.25 * (1.0 - r.s22);
    return r;
}

int q_of(int d) { return (d >= 1 && d <= 4) ? 1 + 2 * d * d : 0; }

// Largest eps for which the scheme is accepted.  d = 3, 4: w1 = 1/6 - (d-1) eps/3
// must stay >= 0; beyond it the von Neumann spectral radius exceeds 1.  d = 2:
// the spectral radius stays 1 up to eps ~ 0.486 (w1 > 0 up to 0.5); 0.48 is
// accepted.  d = 1: stable for every eps tried.
double eps_limit(int d) {
    switch (d) {
        case 2: return 0.48;
        case 3: return 0.25;
        case 4: return 1.0 / 6.0;
        default: return INFINITY;
    }
}

lb_status validate(const lb_config* c) {
    if (!c) return fail(LB_ERR_INVALID_ARG, "config is NULL");
    if (c->dim < 1 || c->dim > 4) return fail(LB_ERR_INVALID_ARG, "dim must be 1, 2, 3 or 4");
    if (c->flags & ~LB_FLAG_BOUNDED) return fail(LB_ERR_INVALID_ARG, "unknown flags");
    if ((c->flags & LB_FLAG_BOUNDED) && (c->dim != 1 || c->n[0] < 2))
        return fail(LB_ERR_INVALID_ARG, "LB_FLAG_BOUNDED needs dim = 1 and n[0] >= 2");
    int64_t V = 1;
    for (int a = 0; a < 4; ++a) {
        if (c->n[a] < 1) return fail(LB_ERR_INVALID_ARG, "every n[a] must be >= 1");
        if (a >= c->dim && c->n[a] != 1)
            return fail(LB_ERR_INVALID_ARG, "n[a] must be 1 for a >= dim");
        if (c->n[a] > INT_MAX) return fail(LB_ERR_INVALID_ARG, "n[a] too large");
        V *= c->n[a];
        if (V > (int64_t)INT_MAX) return fail(LB_ERR_INVALID_ARG, "more than 2^31-1 nodes");
    }
    if (c->dim >= 2 && (c->n[1] + lbm::BLOCK_Y - 1) / lbm::BLOCK_Y > 65535)
        return fail(LB_ERR_INVALID_ARG, "n[1] exceeds the launch-grid limit");
    if (c->dim >= 3 && c->n[2] * c->n[3] > 65535)
        return fail(LB_ERR_INVALID_ARG, "n[2]*n[3] exceeds the launch-grid limit");
    if (!(c->dx > 0) || !(c->dt > 0) || !(c->nu > 0) || !std::isfinite(c->dx) ||
        !std::isfinite(c->dt) || !std::isfinite(c->nu))
        return fail(LB_ERR_INVALID_ARG, "dx, dt and nu must be finite and > 0");
    const double eps = c->nu * c->dt / (c->dx * c->dx);
    if (!std::isfinite(eps) || !(eps > 0)) return fail(LB_ERR_INVALID_ARG, "eps is not finite");
    if (eps > eps_limit(c->dim))
        return fail(LB_ERR_UNSTABLE, "eps = nu dt/dx^2 exceeds the stability limit of the lattice "
                                     "(D2Q9 0.48, D3Q19 1/4, D4Q33 1/6)");
    return LB_OK;
}

Geo make_geo(const lb_config* c) {
    Geo g;
    g.nx = (int)c->n[0];
    g.ny = (int)c->n[1];
    g.nz = (int)c->n[2];
    g.nw = (int)c->n[3];
    g.V = (int64_t)g.nx * g.ny * g.nz * g.nw;
    return g;
}

// Elements of one state buffer: q populations of every node, V rounded up to
// whole chunks.
int64_t elements_of(const lb_config* c) {
    return (int64_t)q_of(c->dim) * lbm::chunks_of(make_geo(c).V) * lbm::CHUNK;
}

}  // namespace

// Fixed device array behind lb_adjoint_segment_static: the partials tables
// of one checkpoint segment.  Every GPU the library runs on holds its own
// copy for the life of the process.  In host code `scratch` names a host-side
// stand-in, not device memory: its device address comes from
// hipGetSymbolAddress, taken once per device (scratch_address) and used
// everywhere host code needs the array.
static __device__ __align__(256) double scratch[LB_SEGMENT_SCRATCH_DOUBLES];

namespace {

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_addr;  // device ordinal -> address of its copy

// Address of the current device's copy of `scratch` (looked up once per device).
lb_status scratch_address(double** out) {
    *out = nullptr;
    int dev = -1;
    LB_HIP(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it == g_scratch_addr.end()) {
        void* p = nullptr;
        LB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        it = g_scratch_addr.emplace(dev, static_cast<double*>(p)).first;
    }
    *out = it->second;
    return LB_OK;
}

}  // namespace

struct lb_solver {
    lb_config cfg;
    int d, q;
    Geo g;
    Rates r;
    hipStream_t stream;
    double* buf[2];
    int cur;
    int64_t steps;
    bool inited;
    double* partials;
    int64_t npartials;
    int* flag;
    int steps_per_pass;  // LB_OPT_STEPS_PER_PASS: 1, 2, 4 or 8
    int64_t check_interval;  // LB_OPT_CHECK_INTERVAL: 0 (off) or steps between state checks
    int64_t since_check;     // steps lb_step has run since the last state check
    bool twin_ok;            // the current state was written by a collision (twins equal)
    bool bounded;        // LB_FLAG_BOUNDED
    double* wall_now;    // bounded: theta at the two end nodes at the current time
    double* seg_partials;  // lb_adjoint_segment: one partials table per launch
    int64_t seg_cap;       // doubles seg_partials holds
    double* scratch;       // this device's copy of `scratch` (lb_adjoint_segment_static)
};

// Make s->seg_partials hold at least n doubles.
static lb_status reserve_seg_partials(lb_solver* s, int64_t n) {
    if (n <= s->seg_cap) return LB_OK;
    if (s->seg_partials) (void)hipFree(s->seg_partials);
    s->seg_partials = nullptr;
    s->seg_cap = 0;
    LB_HIP(hipMalloc((void**)&s->seg_partials, sizeof(double) * (size_t)n),
           "hipMalloc segment partials");
    s->seg_cap = n;
    return LB_OK;
}

static lb_status not_bounded(const lb_solver* s, const char* what) {
    if (s->bounded) return fail(LB_ERR_STATE, what);
    return LB_OK;
}

extern "C" {

const char* lb_last_error(void) { return g_err.c_str(); }

int32_t lb_num_populations(int32_t dim) { return q_of(dim); }

lb_status lb_parameters(const lb_config* cfg, double* out7) {
    lb_status st = validate(cfg);
    if (st == LB_ERR_UNSTABLE) st = LB_OK;  // parameters are defined for any eps > 0
    if (st != LB_OK) return st;
    if (!out7) return fail(LB_ERR_INVALID_ARG, "out is NULL");
    const Rates r = make_rates(cfg->dim, cfg->dx, cfg->dt, cfg->nu);
    out7[0] = r.eps;
    out7[1] = r.s1;
    out7[2] = r.s21;
    out7[3] = r.s22;
    out7[4] = r.w0;
    out7[5] = r.w1;
    out7[6] = r.wd;
    return LB_OK;
}

int64_t lb_state_elements(const lb_config* cfg) {
    if (validate(cfg) == LB_ERR_INVALID_ARG) return 0;
    return elements_of(cfg);
}

size_t lb_state_bytes(const lb_config* cfg) {
    if (validate(cfg) == LB_ERR_INVALID_ARG) return 0;
    return (size_t)elements_of(cfg) * sizeof(double);
}

int64_t lb_state_chunk(void) { return lbm::CHUNK; }

lb_status lb_create(const lb_config* cfg, void* hip_stream, double* f_a, double* f_b,
                    lb_solver** out) {
    if (!out) return fail(LB_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    lb_status st = validate(cfg);
    if (st != LB_OK) return st;
    if (!f_a || !f_b) return fail(LB_ERR_INVALID_ARG, "state buffers must not be NULL");
    const size_t bytes = lb_state_bytes(cfg);
    const char* a = (const char*)f_a;
    const char* b = (const char*)f_b;
    if (a < b + bytes && b < a + bytes) return fail(LB_ERR_INVALID_ARG, "f_a and f_b overlap");
    lb_solver* s = new (std::nothrow) lb_solver();
    if (!s) return fail(LB_ERR_OOM, "host allocation failed");
    s->cfg = *cfg;
    s->d = cfg->dim;
    s->q = q_of(cfg->dim);
    s->g = make_geo(cfg);
    s->r = make_rates(cfg->dim, cfg->dx, cfg->dt, cfg->nu);
    s->stream = (hipStream_t)hip_stream;
    s->buf[0] = f_a;
    s->buf[1] = f_b;
    s->cur = 0;
    s->steps = 0;
    s->inited = false;
    s->steps_per_pass = lbm::MAX_STEPS_PER_PASS;
    s->check_interval = 0;
    s->since_check = 0;
    s->twin_ok = false;
    s->npartials = lbm::launch_shape(s->d, s->g).nblocks;
    s->partials = nullptr;
    s->flag = nullptr;
    s->bounded = (cfg->flags & LB_FLAG_BOUNDED) != 0;
    s->wall_now = nullptr;
    s->seg_partials = nullptr;
    s->seg_cap = 0;
    s->scratch = nullptr;
    // set-up of lb_adjoint_segment_static: the device copy of the scratch
    // array of the device current at creation (the solver's device)
    lb_status sst = scratch_address(&s->scratch);
    if (sst != LB_OK) {
        delete s;
        return sst;
    }
    hipError_t e = hipMalloc((void**)&s->partials, sizeof(double) * (size_t)s->npartials);
    if (e == hipSuccess) e = hipMalloc((void**)&s->flag, sizeof(int));
    if (e == hipSuccess && s->bounded) e = hipMalloc((void**)&s->wall_now, 2 * sizeof(double));
    if (e != hipSuccess) {
        if (s->partials) (void)hipFree(s->partials);
        if (s->flag) (void)hipFree(s->flag);
        delete s;
        return hip_fail(e, "hipMalloc of solver tables");
    }
    *out = s;
    return LB_OK;
}

lb_status lb_destroy(lb_solver* s) {
    if (!s) return LB_OK;
    if (s->partials) (void)hipFree(s->partials);
    if (s->flag) (void)hipFree(s->flag);
    if (s->wall_now) (void)hipFree(s->wall_now);
    if (s->seg_partials) (void)hipFree(s->seg_partials);
    delete s;
    return LB_OK;
}

static lb_status check_theta(lb_solver* s, const double* theta, int64_t n) {
    LB_HIP(hipMemsetAsync(s->flag, 0, sizeof(int), s->stream), "hipMemsetAsync");
    LB_HIP(lbm::launch_check_theta(theta, n, s->flag, s->stream), "check_theta launch");
    int h = 0;
    LB_HIP(hipMemcpyAsync(&h, s->flag, sizeof(int), hipMemcpyDeviceToHost, s->stream),
           "hipMemcpyAsync");
    LB_HIP(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    if (h) return fail(LB_ERR_NONFINITE, "theta0 must be finite and > 0 (Cole-Hopf)");
    return LB_OK;
}

// LB_OPT_CHECK_INTERVAL: after `steps` more steps, check the current state
// once the interval is reached (synchronises the stream).
static lb_status after_steps(lb_solver* s, int64_t steps) {
    if (s->check_interval <= 0) return LB_OK;
    s->since_check += steps;
    if (s->since_check < s->check_interval) return LB_OK;
    s->since_check = 0;
    LB_HIP(hipMemsetAsync(s->flag, 0, sizeof(int), s->stream), "hipMemsetAsync");
    LB_HIP(lbm::launch_check_state(s->d, s->g, s->buf[s->cur], s->flag, s->stream),
           "check_state launch");
    int h = 0;
    LB_HIP(hipMemcpyAsync(&h, s->flag, sizeof(int), hipMemcpyDeviceToHost, s->stream),
           "hipMemcpyAsync");
    LB_HIP(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    if (h)
        return fail(LB_ERR_NONFINITE, "theta is not finite and positive at some node after step " +
                                          std::to_string((long long)s->steps));
    return LB_OK;
}

lb_status lb_init(lb_solver* s, const double* theta0, const double* grad_theta0,
                  int32_t check) {
    if (!s || !theta0) return fail(LB_ERR_INVALID_ARG, "solver and theta0 must not be NULL");
    if (s->bounded && !grad_theta0)
        return fail(LB_ERR_INVALID_ARG, "a bounded interval needs grad_theta0");
    if (check) {
        lb_status st = check_theta(s, theta0, s->g.V);
        if (st != LB_OK) return st;
    }
    LB_HIP(lbm::launch_init(s->d, s->g, s->r, theta0, grad_theta0, s->buf[0], s->stream),
           "init launch");
    if (s->bounded) {
        LB_HIP(hipMemcpyAsync(s->wall_now, theta0, sizeof(double), hipMemcpyDeviceToDevice,
                              s->stream),
               "hipMemcpyAsync");
        LB_HIP(hipMemcpyAsync(s->wall_now + 1, theta0 + (s->g.nx - 1), sizeof(double),
                              hipMemcpyDeviceToDevice, s->stream),
               "hipMemcpyAsync");
    }
    s->cur = 0;
    s->steps = 0;
    s->since_check = 0;
    s->twin_ok = false;
    s->inited = true;
    return LB_OK;
}

lb_status lb_step(lb_solver* s, int64_t nsteps) {
    if (!s) return fail(LB_ERR_INVALID_ARG, "solver is NULL");
    if (nsteps < 0) return fail(LB_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (!s->inited) return fail(LB_ERR_STATE, "lb_step before lb_init/lb_set_state");
    if (s->bounded) return fail(LB_ERR_STATE, "a bounded interval steps with lb_step_bounded");
    if (s->d == 1 && s->g.nx <= lbm::RESIDENT_MAX_1D && nsteps >= 2) {
        // whole run in one launch; the result lands where the per-step
        // ping-pong would have left it
        const int dst = s->cur ^ (int)(nsteps & 1);
        LB_HIP(lbm::launch_step_resident1(s->g, s->r, s->buf[s->cur], s->buf[dst], nsteps,
                                          nullptr, nullptr, s->stream),
               "resident step launch");
        s->cur = dst;
        s->steps += nsteps;
        return after_steps(s, nsteps);
    }
    // Launch plan: on D2Q9 passes of 8, 4 and 2 steps (within the limit),
    // on D3Q19 passes of 2, then single steps, as runs (steps per launch,
    // launches).  A state written by a collision holds equal twin
    // populations (twin<D>, lbm_lattice.h), so a launch reads only the
    // independent ones unless the state came from lb_init or lb_set_state,
    // and every launch but the last writes only those; the last launch, and
    // any launch whose state is checked (LB_OPT_CHECK_INTERVAL), writes all
    // q, so the state a call leaves (the one every other call sees) is
    // complete.
    std::vector<std::pair<int, int64_t>> runs;
    {
        int64_t n = 0;
        if (s->d == 2) {
            for (int pass = s->steps_per_pass; pass >= 2; pass /= 2) {
                const int64_t k = (nsteps - n) / pass;
                if (k > 0) runs.emplace_back(pass, k);
                n += k * pass;
            }
        } else if (s->d == 3 && s->steps_per_pass >= lbm::MAX_STEPS_PER_PASS_3D) {
            const int pass = lbm::MAX_STEPS_PER_PASS_3D;
            const int64_t k = (nsteps - n) / pass;
            if (k > 0) runs.emplace_back(pass, k);
            n += k * pass;
        }
        if (n < nsteps) runs.emplace_back(1, nsteps - n);
    }
    lb_status st = LB_OK;
    for (size_t ri = 0; ri < runs.size(); ++ri) {
        const int steps = runs[ri].first;
        for (int64_t t = 0; t < runs[ri].second; ++t) {
            const bool last = ri + 1 == runs.size() && t + 1 == runs[ri].second;
            const bool checked =
                s->check_interval > 0 && s->since_check + steps >= s->check_interval;
            const bool rin = s->twin_ok;
            const bool wout = !last && !checked;
            const double* src = s->buf[s->cur];
            double* dst = s->buf[1 - s->cur];
            if (steps == 1)
                LB_HIP(lbm::launch_step(s->d, s->g, s->r, src, dst, s->stream, rin, wout),
                       "step launch");
            else if (s->d == 2)
                LB_HIP(lbm::launch_steps(steps, s->g, s->r, src, dst, s->stream, rin, wout),
                       "multi-step launch");
            else
                LB_HIP(lbm::launch_steps3(steps, s->g, s->r, src, dst, s->stream, rin, wout),
                       "multi-step launch");
            s->cur ^= 1;
            s->steps += steps;
            s->twin_ok = true;
            if ((st = after_steps(s, steps)) != LB_OK) return st;
        }
    }
    return LB_OK;
}

lb_status lb_step_bounded(lb_solver* s, int64_t nsteps, const double* walls) {
    if (!s) return fail(LB_ERR_INVALID_ARG, "solver is NULL");
    if (!s->bounded) return fail(LB_ERR_STATE, "the solver was not created with LB_FLAG_BOUNDED");
    if (nsteps < 0) return fail(LB_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (!s->inited) return fail(LB_ERR_STATE, "lb_step_bounded before lb_init/lb_set_state");
    if (nsteps == 0) return LB_OK;
    if (!walls) return fail(LB_ERR_INVALID_ARG, "walls is NULL");
    if (s->g.nx <= lbm::RESIDENT_MAX_1D) {
        const int dst = s->cur ^ (int)(nsteps & 1);
        LB_HIP(lbm::launch_step_resident1(s->g, s->r, s->buf[s->cur], s->buf[dst], nsteps, walls,
                                          s->wall_now, s->stream),
               "resident step launch");
        s->cur = dst;
    } else {
        for (int64_t n = 0; n < nsteps; ++n) {
            const double* wall = n == 0 ? s->wall_now : walls + 2 * (n - 1);
            LB_HIP(lbm::launch_step_wall1(s->g, s->r, s->buf[s->cur], s->buf[1 - s->cur], wall,
                                          s->stream),
                   "step launch");
            s->cur ^= 1;
        }
        LB_HIP(hipMemcpyAsync(s->wall_now, walls + 2 * (nsteps - 1), 2 * sizeof(double),
                              hipMemcpyDeviceToDevice, s->stream),
               "hipMemcpyAsync");
    }
    s->steps += nsteps;
    return LB_OK;
}

lb_status lb_set_option(lb_solver* s, int32_t option, int32_t value) {
    if (!s) return fail(LB_ERR_INVALID_ARG, "solver is NULL");
    switch (option) {
        case LB_OPT_STEPS_PER_PASS: {
            int p = 1;
            while (p * 2 <= value && p * 2 <= lbm::MAX_STEPS_PER_PASS) p *= 2;
            s->steps_per_pass = p;
            return LB_OK;
        }
        case LB_OPT_CHECK_INTERVAL:
            if (value < 0) return fail(LB_ERR_INVALID_ARG, "the check interval must be >= 0");
            s->check_interval = value;
            s->since_check = 0;
            return LB_OK;
        default:
            return fail(LB_ERR_INVALID_ARG, "unknown option");
    }
}

lb_status lb_step_buffers(lb_solver* s, const double* src, double* dst) {
    if (!s || !src || !dst) return fail(LB_ERR_INVALID_ARG, "NULL argument");
    if (src == dst) return fail(LB_ERR_INVALID_ARG, "src and dst must differ");
    lb_status st = not_bounded(s, "lb_step_buffers is periodic only");
    if (st != LB_OK) return st;
    LB_HIP(lbm::launch_step(s->d, s->g, s->r, src, dst, s->stream), "step launch");
    return LB_OK;
}

double* lb_current_state(const lb_solver* s) { return s ? s->buf[s->cur] : nullptr; }
int64_t lb_steps_taken(const lb_solver* s) { return s ? s->steps : -1; }

lb_status lb_macro_buffer(lb_solver* s, const double* state, double* theta, double* u,
                          double* grad_theta) {
    if (!s || !state) return fail(LB_ERR_INVALID_ARG, "NULL argument");
    lb_status st = not_bounded(s, "lb_macro_buffer is periodic only (use lb_macro)");
    if (st != LB_OK) return st;
    if (!theta && !u && !grad_theta) return LB_OK;
    LB_HIP(lbm::launch_macro(s->d, s->g, s->r, state, theta, u, grad_theta, s->stream),
           "macro launch");
    return LB_OK;
}

lb_status lb_macro(lb_solver* s, double* theta, double* u, double* grad_theta) {
    if (!s) return fail(LB_ERR_INVALID_ARG, "solver is NULL");
    if (!s->inited) return fail(LB_ERR_STATE, "lb_macro before lb_init/lb_set_state");
    if (s->bounded) {
        if (!theta && !u && !grad_theta) return LB_OK;
        LB_HIP(lbm::launch_macro_wall1(s->g, s->r, s->buf[s->cur], theta, u, grad_theta,
                                       s->wall_now, s->stream),
               "macro launch");
        return LB_OK;
    }
    return lb_macro_buffer(s, s->buf[s->cur], theta, u, grad_theta);
}

lb_status lb_get_state(lb_solver* s, double* f_out) {
    if (!s || !f_out) return fail(LB_ERR_INVALID_ARG, "NULL argument");
    if (!s->inited) return fail(LB_ERR_STATE, "no state yet");
    if (s->bounded)
        LB_HIP(lbm::launch_get_state_wall1(s->g, s->buf[s->cur], f_out, s->wall_now, s->stream),
               "get_state");
    else
        LB_HIP(lbm::launch_get_state(s->d, s->g, s->buf[s->cur], f_out, s->stream), "get_state");
    return LB_OK;
}

lb_status lb_set_state(lb_solver* s, const double* f_in, int64_t step) {
    if (!s || !f_in) return fail(LB_ERR_INVALID_ARG, "NULL argument");
    if (step < 0) return fail(LB_ERR_INVALID_ARG, "step must be >= 0");
    LB_HIP(lbm::launch_set_state(s->d, s->g, f_in, s->buf[0], s->stream), "set_state");
    if (s->bounded)
        LB_HIP(lbm::launch_wall_from_dense1(s->g, f_in, s->wall_now, s->stream), "set_state walls");
    s->cur = 0;
    s->steps = step;
    s->since_check = 0;
    s->twin_ok = false;
    s->inited = true;
    return LB_OK;
}

lb_status lb_layout_from_dense(lb_solver* s, const double* dense, double* buf) {
    if (!s || !dense || !buf) return fail(LB_ERR_INVALID_ARG, "NULL argument");
    LB_HIP(lbm::launch_layout_from_dense(s->d, s->g, dense, buf, s->stream), "layout_from_dense");
    return LB_OK;
}

lb_status lb_layout_to_dense(lb_solver* s, const double* buf, double* dense) {
    if (!s || !dense || !buf) return fail(LB_ERR_INVALID_ARG, "NULL argument");
    LB_HIP(lbm::launch_layout_to_dense(s->d, s->g, buf, dense, s->stream), "layout_to_dense");
    return LB_OK;
}

lb_status lb_theta_from_velocity(lb_solver* s, const double* u0, double* theta0, double* grad) {
    if (!s || !u0 || !theta0) return fail(LB_ERR_INVALID_ARG, "NULL argument");
    lb_status st = not_bounded(s, "lb_theta_from_velocity is periodic only");
    if (st != LB_OK) return st;
    const int64_t nw = lbm::potential_workspace(s->d, s->g);
    double* work = nullptr;
    LB_HIP(hipMalloc((void**)&work, sizeof(double) * (size_t)nw), "hipMalloc potential workspace");
    hipError_t e = lbm::launch_theta_from_velocity(s->d, s->g, s->cfg.dx, s->cfg.nu, u0, work,
                                                   theta0, grad, s->stream);
    hipError_t e2 = hipStreamSynchronize(s->stream);
    (void)hipFree(work);
    if (e != hipSuccess) return hip_fail(e, "theta_from_velocity launch");
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamSynchronize");
    return LB_OK;
}

lb_status lb_macro_adjoint(lb_solver* s, const double* state, const double* g_theta,
                           const double* g_u, double* lambda, double* g_eps) {
    if (!s || !state || !lambda || !g_eps) return fail(LB_ERR_INVALID_ARG, "NULL argument");
    lb_status st = not_bounded(s, "the adjoint is periodic only");
    if (st != LB_OK) return st;
    LB_HIP(lbm::launch_macro_adjoint(s->d, s->g, s->r, state, g_theta, g_u, lambda, s->partials,
                                     s->stream),
           "macro_adjoint launch");
    LB_HIP(lbm::launch_finalize(s->partials, s->npartials, g_eps, s->stream), "finalize");
    return LB_OK;
}

lb_status lb_adjoint_step(lb_solver* s, const double* state_n, const double* lambda_in,
                          double* lambda_out, double* g_eps) {
    if (!s || !state_n || !lambda_in || !lambda_out || !g_eps)
        return fail(LB_ERR_INVALID_ARG, "NULL argument");
    if (lambda_in == lambda_out) return fail(LB_ERR_INVALID_ARG, "lambda_in == lambda_out");
    lb_status st = not_bounded(s, "the adjoint is periodic only");
    if (st != LB_OK) return st;
    LB_HIP(lbm::launch_adjoint_step(s->d, s->g, s->r, state_n, lambda_in, lambda_out, s->partials,
                                    s->npartials, s->stream),
           "adjoint_step launch");
    LB_HIP(lbm::launch_finalize(s->partials, s->npartials, g_eps, s->stream), "finalize");
    return LB_OK;
}

}  // extern "C"

// Launch plan of one checkpoint segment: the reverse passes and the size of
// the partials tables they write (one table per launch plus one sum each).
struct SegmentPlan {
    std::vector<int> reverse;  // D2Q9: adjoint steps per launch, in launch order
    int64_t T = 0;             // doubles per table
    int64_t ntables = 0;
    int64_t doubles() const { return ntables * (T + 1); }
};

static SegmentPlan segment_plan(const lb_solver* s, int64_t m) {
    SegmentPlan p;
    if (s->d == 2) {
        // reverse sweep in passes of up to steps_per_pass (at most 4) adjoint
        // steps over n0+m-1 .. n0+1, then the step at the checkpoint
        int64_t left = m - 1;
        for (int pass = std::min(s->steps_per_pass, lbm::MAX_ADJOINT_STEPS_PER_PASS); pass >= 1;
             pass /= 2)
            for (; left >= pass; left -= pass) p.reverse.push_back(pass);
        p.reverse.push_back(1);
        p.T = std::max(lbm::adjoint_steps_table(s->g), s->npartials);
        p.ntables = (int64_t)p.reverse.size();
    } else {
        p.T = s->npartials;
        p.ntables = m;
    }
    return p;
}

// One checkpoint segment (lb_adjoint_segment); `tables` holds plan.doubles()
// doubles, every one of which the launches write before it is read.
static lb_status run_segment(lb_solver* s, const SegmentPlan& plan, const double* ckpt, int64_t m,
                             double* work, double* lambda, double* lambda_tmp, double* g_eps,
                             double* tables) {
    const int64_t se = elements_of(&s->cfg);
    // forward recomputation of the segment's states f^{n0+1} .. f^{n0+m-1}
    // (bitwise single steps): on D2Q9 by multi-step passes that store the
    // state after each of their steps, the rest one step at a time.  Every
    // state in work comes from a collision, so its twin populations are not
    // stored and are read from their partners' planes; the checkpoint may be
    // any state and is read whole.
    const double* prev = ckpt;
    int64_t j = 1;  // next state to produce
    if (s->d == 2) {
        for (int pass = s->steps_per_pass; pass >= 2; pass /= 2) {
            for (; j + pass <= m; j += pass) {
                double* out = work + (j - 1) * se;
                LB_HIP(lbm::launch_steps_all(pass, s->g, s->r, prev, out, se, s->stream,
                                             prev != ckpt, true),
                       "multi-step launch");
                prev = out + (int64_t)(pass - 1) * se;
            }
        }
    }
    for (; j < m; ++j) {
        double* nxt = work + (j - 1) * se;
        LB_HIP(lbm::launch_step(s->d, s->g, s->r, prev, nxt, s->stream, prev != ckpt, true),
               "step launch");
        prev = nxt;
    }
    double* lin = lambda;
    double* lout = lambda_tmp;
    const int64_t T = plan.T, nt = plan.ntables;
    if (s->d == 2) {
        // the states of n0+m-1 .. n0+1 are consecutive in work; every launch
        // leaves a full table of T partials
        int64_t N = m;  // lin holds lambda^{n0+N}
        for (int64_t t = 0; t < nt; ++t) {
            const double* ftop = N == 1 ? ckpt : work + (N - 2) * se;  // f^{n0+N-1}
            const int steps = plan.reverse[(size_t)t];
            if (steps == 1)
                LB_HIP(lbm::launch_adjoint_step(2, s->g, s->r, ftop, lin, lout, tables + t * T, T,
                                                s->stream, N != 1),
                       "adjoint_step launch");
            else  // reads f^{n0+N-1} .. f^{n0+N-steps}, all in work (N > steps)
                LB_HIP(lbm::launch_adjoint_steps(steps, s->g, s->r, lin, lout, ftop, se,
                                                 tables + t * T, T, s->stream, true),
                       "adjoint multi-step launch");
            std::swap(lin, lout);
            N -= steps;
        }
    } else {
        // one adjoint step per launch; step j leaves its block partials in
        // table j, and one reduction adds the tables in the order of the steps
        for (j = m - 1; j >= 0; --j) {
            const double* fn = j == 0 ? ckpt : work + (j - 1) * se;
            LB_HIP(lbm::launch_adjoint_step(s->d, s->g, s->r, fn, lin, lout, tables + j * T, T,
                                            s->stream, j != 0),
                   "adjoint_step launch");
            std::swap(lin, lout);
        }
    }
    LB_HIP(lbm::launch_finalize_tables(tables, T, nt, tables + nt * T, g_eps, s->stream),
           "finalize");
    if (lin != lambda)
        LB_HIP(hipMemcpyAsync(lambda, lin, sizeof(double) * (size_t)se, hipMemcpyDeviceToDevice,
                              s->stream),
               "hipMemcpyAsync");
    return LB_OK;
}

static lb_status check_segment_args(lb_solver* s, const double* ckpt, int64_t m,
                                    const double* lambda, const double* lambda_tmp,
                                    const double* g_eps) {
    if (!s || !ckpt || !lambda || !lambda_tmp || !g_eps)
        return fail(LB_ERR_INVALID_ARG, "NULL argument");
    if (m < 0) return fail(LB_ERR_INVALID_ARG, "m must be >= 0");
    if (lambda == lambda_tmp) return fail(LB_ERR_INVALID_ARG, "lambda == lambda_tmp");
    return not_bounded(s, "the adjoint is periodic only");
}

extern "C" {

lb_status lb_adjoint_segment(lb_solver* s, const double* ckpt, int64_t m, double* work,
                             double* lambda, double* lambda_tmp, double* g_eps) {
    lb_status st = check_segment_args(s, ckpt, m, lambda, lambda_tmp, g_eps);
    if (st != LB_OK) return st;
    if (m > 1 && !work) return fail(LB_ERR_INVALID_ARG, "work is NULL");
    if (m == 0) return LB_OK;
    const SegmentPlan plan = segment_plan(s, m);
    st = reserve_seg_partials(s, plan.doubles());
    if (st != LB_OK) return st;
    return run_segment(s, plan, ckpt, m, work, lambda, lambda_tmp, g_eps, s->seg_partials);
}

lb_status lb_adjoint_segment_static(lb_solver* s, const double* ckpt, int64_t m, double* work,
                                    double* lambda, double* lambda_tmp, double* g_eps) {
    lb_status st = check_segment_args(s, ckpt, m, lambda, lambda_tmp, g_eps);
    if (st != LB_OK) return st;
    if (m == 0) return LB_OK;
    const SegmentPlan plan = segment_plan(s, m);
    if (plan.doubles() > LB_SEGMENT_SCRATCH_DOUBLES)
        return fail(LB_ERR_INVALID_ARG,
                    "segment needs " + std::to_string(plan.doubles()) +
                        " doubles of partials, more than the fixed scratch array holds (" +
                        std::to_string((long long)LB_SEGMENT_SCRATCH_DOUBLES) +
                        "): use lb_adjoint_segment or a shorter segment");
    if (m > 1 && !work) return fail(LB_ERR_INVALID_ARG, "work is NULL");
    if (!s->scratch) return fail(LB_ERR_STATE, "no scratch address for this solver's device");
    return run_segment(s, plan, ckpt, m, work, lambda, lambda_tmp, g_eps, s->scratch);
}

lb_status lb_init_adjoint(lb_solver* s, const double* theta0, const double* grad_theta0,
                          const double* lambda0, double* g_theta0, double* g_grad,
                          double* g_eps, double* g_nu) {
    if (!s || !theta0 || !lambda0 || !g_theta0 || !g_eps)
        return fail(LB_ERR_INVALID_ARG, "NULL argument");
    if (g_nu == g_eps) return fail(LB_ERR_INVALID_ARG, "g_nu and g_eps must differ");
    lb_status st = not_bounded(s, "the adjoint is periodic only");
    if (st != LB_OK) return st;
    LB_HIP(lbm::launch_init_adjoint(s->d, s->g, s->r, theta0, grad_theta0, lambda0, g_theta0,
                                    g_grad, s->partials, s->stream),
           "init_adjoint launch");
    // eps = nu dt / dx^2, so dL/dnu = (dt / dx^2) dL/deps
    const double nu_scale = s->cfg.dt / (s->cfg.dx * s->cfg.dx);
    LB_HIP(lbm::launch_finalize(s->partials, s->npartials, g_eps, s->stream, g_nu, nu_scale),
           "finalize");
    return LB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------

// Tile mode of a new batch: 8-step tiles of 64 rows (autotuning may change it).
constexpr int kDefaultPassSteps = 8;
constexpr int kDefaultStripRows = 64;

struct lb_batch {
    std::vector<lb_config> cfgs;
    std::vector<int64_t> offsets, elems, node_offsets;
    std::vector<BatchInst> insts;
    hipStream_t stream;
    hipStream_t capture;
    double* pool[2];
    int64_t pool_elems;
    int cur;
    int64_t steps;
    bool inited;
    bool twin_ok;  // pool[cur] was written by a collision (twins equal their partners)
    BatchInst* d_insts;
    BatchTile* d_tiles;
    int64_t ntiles;
    BatchTile* d_lin;  // linear tiles, for the steps a multi-step mode leaves over
    int64_t nlin;
    int tx, ty;
    bool off32;  // every instance's state is under 4 GiB
    // graphs keyed by (step count, starting pool, twin_ok)
    std::map<std::tuple<int64_t, int, bool>, hipGraphExec_t> graphs;
};

// Multi-step tile modes: tx = -S (two-wave LDS strips of
// batch_strip_width(S) columns) or tx = -16 - S (one-wave strips of
// strip_width(S) columns), S = 2, 4, 8.
constexpr int kOneWaveMode = 16;
static bool mode_multi_step(int tx) { return tx < 0; }
static bool mode_one_wave(int tx) { return tx < -kOneWaveMode; }
static int mode_steps(int tx) { return mode_one_wave(tx) ? -tx - kOneWaveMode : -tx; }
static int mode_width(int tx) {
    return mode_one_wave(tx) ? lbm::strip_width(mode_steps(tx))
                             : lbm::batch_strip_width(mode_steps(tx));
}

static void drop_graphs(lb_batch* b) {
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
}

// Graphs kept per batch (one per step count, starting pool and twin_ok); a new one
// beyond this clears the cache once the work already enqueued has finished.
constexpr size_t kMaxCachedGraphs = 16;

// Tile tables.  tx == 0: 256 consecutive node indices of one instance;
// multi-step modes: S-step tiles of mode_width(tx) columns x ty rows (y1 in
// .pad), ordered strip-fastest within an instance so that neighbouring strips
// share an XCD; otherwise tx x ty rectangles.
static std::vector<BatchTile> tile_list(const lb_batch* b, int tx, int ty) {
    std::vector<BatchTile> tiles;
    for (size_t i = 0; i < b->insts.size(); ++i) {
        const BatchInst& in = b->insts[i];
        if (tx == 0) {
            const int64_t V = (int64_t)in.nx * in.ny;
            for (int64_t k0 = 0; k0 < V; k0 += 256) tiles.push_back(BatchTile{(int)i, (int)k0, 0, 0});
        } else if (mode_multi_step(tx)) {
            for (int y0 = 0; y0 < in.ny; y0 += ty)
                for (int x0 = 0; x0 < in.nx; x0 += mode_width(tx))
                    tiles.push_back(BatchTile{(int)i, x0, y0, std::min(y0 + ty, in.ny)});
        } else {
            for (int y0 = 0; y0 < in.ny; y0 += ty)
                for (int x0 = 0; x0 < in.nx; x0 += tx) tiles.push_back(BatchTile{(int)i, x0, y0, 0});
        }
    }
    return tiles;
}

static lb_status upload_tiles(const std::vector<BatchTile>& tiles, BatchTile** d, int64_t* n) {
    if (tiles.size() > (size_t)INT_MAX) return fail(LB_ERR_INVALID_ARG, "too many tiles");
    if (*d) (void)hipFree(*d);
    *d = nullptr;
    *n = 0;
    if (!tiles.empty()) {
        LB_HIP(hipMalloc((void**)d, sizeof(BatchTile) * tiles.size()), "hipMalloc tiles");
        LB_HIP(hipMemcpy(*d, tiles.data(), sizeof(BatchTile) * tiles.size(), hipMemcpyHostToDevice),
               "hipMemcpy tiles");
    }
    *n = (int64_t)tiles.size();
    return LB_OK;
}

static lb_status build_tiles(lb_batch* b, int tx, int ty) {
    lb_status st = upload_tiles(tile_list(b, tx, ty), &b->d_tiles, &b->ntiles);
    if (st != LB_OK) return st;
    b->tx = tx;
    b->ty = ty;
    drop_graphs(b);
    return LB_OK;
}

extern "C" {

int64_t lb_batch_layout(const lb_config* cfgs, int32_t count, int64_t* offsets,
                        int64_t* elems) {
    if (count < 0 || (count > 0 && !cfgs)) return -1;
    int64_t total = 0;
    for (int32_t i = 0; i < count; ++i) {
        if (validate(&cfgs[i]) == LB_ERR_INVALID_ARG || cfgs[i].dim != 2) return -1;
        const int64_t e = elements_of(&cfgs[i]);
        if (offsets) offsets[i] = total;
        if (elems) elems[i] = e;
        total += e;
    }
    return total;
}

lb_status lb_batch_create(const lb_config* cfgs, int32_t count, void* hip_stream,
                          double* pool_a, double* pool_b, lb_batch** out) {
    if (!out) return fail(LB_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1 || !cfgs) return fail(LB_ERR_INVALID_ARG, "need at least one instance");
    for (int32_t i = 0; i < count; ++i) {
        lb_status st = validate(&cfgs[i]);
        if (st != LB_OK) return st;
        if (cfgs[i].dim != 2) return fail(LB_ERR_INVALID_ARG, "batched form is 2-D only");
        if (cfgs[i].flags != 0) return fail(LB_ERR_INVALID_ARG, "batched form is periodic only");
    }
    if (!pool_a || !pool_b || pool_a == pool_b)
        return fail(LB_ERR_INVALID_ARG, "two distinct pools are required");
    lb_batch* b = new (std::nothrow) lb_batch();
    if (!b) return fail(LB_ERR_OOM, "host allocation failed");
    b->cfgs.assign(cfgs, cfgs + count);
    b->offsets.resize(count);
    b->elems.resize(count);
    b->pool_elems = lb_batch_layout(cfgs, count, b->offsets.data(), b->elems.data());
    b->off32 = true;
    for (int32_t i = 0; i < count; ++i)
        if ((uint64_t)b->elems[i] * sizeof(double) > 0xffffffffull) b->off32 = false;
    int64_t nodes = 0;
    for (int32_t i = 0; i < count; ++i) {
        b->node_offsets.push_back(nodes);
        nodes += cfgs[i].n[0] * cfgs[i].n[1];
        BatchInst in;
        in.offset = b->offsets[i];
        in.nx = (int)cfgs[i].n[0];
        in.ny = (int)cfgs[i].n[1];
        in.r = make_rates(2, cfgs[i].dx, cfgs[i].dt, cfgs[i].nu);
        b->insts.push_back(in);
    }
    b->stream = (hipStream_t)hip_stream;
    b->capture = nullptr;
    b->pool[0] = pool_a;
    b->pool[1] = pool_b;
    b->cur = 0;
    b->steps = 0;
    b->inited = false;
    b->twin_ok = false;
    b->d_insts = nullptr;
    b->d_tiles = nullptr;
    b->ntiles = 0;
    b->d_lin = nullptr;
    b->nlin = 0;
    hipError_t e = hipMalloc((void**)&b->d_insts, sizeof(BatchInst) * b->insts.size());
    if (e == hipSuccess)
        e = hipMemcpy(b->d_insts, b->insts.data(), sizeof(BatchInst) * b->insts.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (b->d_insts) (void)hipFree(b->d_insts);
        delete b;
        return hip_fail(e, "batch setup");
    }
    lb_status st = upload_tiles(tile_list(b, 0, 0), &b->d_lin, &b->nlin);
    if (st == LB_OK) st = build_tiles(b, -kDefaultPassSteps, kDefaultStripRows);
    if (st != LB_OK) {
        lb_batch_destroy(b);
        return st;
    }
    *out = b;
    return LB_OK;
}

lb_status lb_batch_destroy(lb_batch* b) {
    if (!b) return LB_OK;
    // graphs and tile tables may still be in use by enqueued work
    (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_lin) (void)hipFree(b->d_lin);
    if (b->d_insts) (void)hipFree(b->d_insts);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
    return LB_OK;
}

lb_status lb_batch_init(lb_batch* b, const double* theta0, const double* grad) {
    if (!b || !theta0) return fail(LB_ERR_INVALID_ARG, "NULL argument");
    for (size_t i = 0; i < b->insts.size(); ++i) {
        const lb_config* c = &b->cfgs[i];
        Geo g = make_geo(c);
        const int64_t no = b->node_offsets[i];
        LB_HIP(lbm::launch_init(2, g, b->insts[i].r, theta0 + no, grad ? grad + 2 * no : nullptr,
                                b->pool[0] + b->offsets[i], b->stream),
               "batch init launch");
    }
    b->cur = 0;
    b->steps = 0;
    b->inited = true;
    b->twin_ok = false;
    return LB_OK;
}

lb_status lb_batch_set_tile(lb_batch* b, int32_t tx, int32_t ty) {
    if (!b) return fail(LB_ERR_INVALID_ARG, "batch is NULL");
    const bool linear = (tx == 0 && ty == 0);
    const int S = mode_steps(tx);
    const bool multi_step = mode_multi_step(tx) && (S == 2 || S == 4 || S == 8) &&
                            (tx == -S || tx == -kOneWaveMode - S) && ty >= 1 && ty <= 65535;
    if (!linear && !multi_step &&
        (tx < 16 || tx > 256 || (tx & (tx - 1)) != 0 || tx * ty != 256))
        return fail(LB_ERR_INVALID_ARG,
                    "tile must be (0,0), (-S, rows) or (-16-S, rows) with S in {2,4,8} and rows "
                    "in [1,65535], or tx*ty = 256 with tx a power of two in [16,256]");
    if (tx == b->tx && ty == b->ty) return LB_OK;
    return build_tiles(b, tx, ty);
}

// Launches that advance nsteps in the current tile mode: passes of S steps
// for a mode (-S, rows), the rest single steps on the linear tiles.
static int64_t batch_launches(const lb_batch* b, int64_t nsteps) {
    if (!mode_multi_step(b->tx)) return nsteps;
    const int S = mode_steps(b->tx);
    return nsteps / S + nsteps % S;
}

// Enqueue nsteps steps starting from pool[cur]; *cur_out receives the pool
// that then holds the state.  As in lb_step, the first launch reads twins
// from their partners' planes when the state came from a collision
// (b->twin_ok), every later launch does, and only the last launch stores the
// twins, so that the pool a call leaves holds a complete state.
static lb_status batch_launch_plain(lb_batch* b, int64_t nsteps, hipStream_t st, int cur,
                                    int* cur_out) {
    const int64_t total = batch_launches(b, nsteps);
    int64_t launch = 0;
    auto io = [&](bool* rin, bool* wout) {
        *rin = launch > 0 || b->twin_ok;
        *wout = launch + 1 < total;
        ++launch;
    };
    bool rin, wout;
    if (mode_multi_step(b->tx)) {
        const int S = mode_steps(b->tx);
        int64_t n = 0;
        for (; n + S <= nsteps; n += S) {
            io(&rin, &wout);
            LB_HIP(lbm::launch_batch_steps(S, b->d_insts, b->d_tiles, b->ntiles, b->pool[cur],
                                           b->pool[1 - cur], b->off32, mode_one_wave(b->tx), st,
                                           rin, wout),
                   "batch multi-step launch");
            cur ^= 1;
        }
        for (; n < nsteps; ++n) {
            io(&rin, &wout);
            LB_HIP(lbm::launch_batch_step(b->d_insts, b->d_lin, b->nlin, 0, 0, b->pool[cur],
                                          b->pool[1 - cur], st, rin, wout),
                   "batch step launch");
            cur ^= 1;
        }
    } else {
        for (int64_t n = 0; n < nsteps; ++n) {
            io(&rin, &wout);
            LB_HIP(lbm::launch_batch_step(b->d_insts, b->d_tiles, b->ntiles, b->tx, b->ty,
                                          b->pool[cur], b->pool[1 - cur], st, rin, wout),
                   "batch step launch");
            cur ^= 1;
        }
    }
    if (cur_out) *cur_out = cur;
    return LB_OK;
}

lb_status lb_batch_step(lb_batch* b, int64_t nsteps, int32_t use_graph) {
    if (!b) return fail(LB_ERR_INVALID_ARG, "batch is NULL");
    if (nsteps < 0) return fail(LB_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (!b->inited) return fail(LB_ERR_STATE, "lb_batch_step before lb_batch_init");
    if (nsteps == 0) return LB_OK;
    int next = b->cur;
    if (!use_graph) {
        lb_status st = batch_launch_plain(b, nsteps, b->stream, b->cur, &next);
        if (st != LB_OK) return st;
    } else {
        auto key = std::make_tuple(nsteps, b->cur, b->twin_ok);
        auto it = b->graphs.find(key);
        if (it == b->graphs.end()) {
            if (b->graphs.size() >= kMaxCachedGraphs) {
                // a cached graph may still be running on the stream
                LB_HIP(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
                drop_graphs(b);
            }
            hipGraph_t graph = nullptr;
            LB_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal),
                   "hipStreamBeginCapture");
            lb_status st = batch_launch_plain(b, nsteps, b->capture, b->cur, nullptr);
            hipError_t e = hipStreamEndCapture(b->capture, &graph);
            if (st != LB_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
            it = b->graphs.emplace(key, exec).first;
        }
        LB_HIP(hipGraphLaunch(it->second, b->stream), "hipGraphLaunch");
        next = b->cur ^ (int)(batch_launches(b, nsteps) & 1);
    }
    b->cur = next;
    b->steps += nsteps;
    b->twin_ok = true;
    return LB_OK;
}

lb_status lb_batch_autotune(lb_batch* b, int32_t steps_per_trial, int32_t* best_tx,
                            int32_t* best_ty) {
    if (!b) return fail(LB_ERR_INVALID_ARG, "batch is NULL");
    if (!b->inited) return fail(LB_ERR_STATE, "autotune needs an initialised batch");
    if (steps_per_trial < 1) steps_per_trial = 1;
    // one-wave strips (-24, rows) favour short segments: on 512 ragged
    // instances 280 GLUPS at 32 rows, 263-264 at 64-192, against 261-263
    // for the two-wave (-8, 128) and (-8, 192)
    static const int cand[][2] = {{0, 0},   {256, 1}, {64, 4},   {16, 16},  {-2, 64},
                                  {-4, 64},  {-8, 32}, {-8, 64},  {-8, 128}, {-8, 192},
                                  {-8, 256}, {-24, 16}, {-24, 32}};
    hipEvent_t e0, e1;
    LB_HIP(hipEventCreate(&e0), "hipEventCreate");
    LB_HIP(hipEventCreate(&e1), "hipEventCreate");
    float best = 1e30f;
    int bx = b->tx, by = b->ty;
    lb_status st = LB_OK;
    for (const auto& c : cand) {
        st = build_tiles(b, c[0], c[1]);
        if (st != LB_OK) break;
        // Trials always launch pool[cur] -> pool[1-cur]: the current state
        // is untouched and the other pool is scratch.  They time the launches
        // a step call runs between its first and its last (twins read from
        // their partners' planes and not stored), whatever pool[cur] holds:
        // what lands in the scratch pool is never read.  Times are per step.
        const int per_launch = mode_multi_step(c[0]) ? mode_steps(c[0]) : 1;
        auto trial = [&](int reps) -> lb_status {
            for (int r = 0; r < reps; ++r) {
                if (mode_multi_step(c[0]))
                    LB_HIP(lbm::launch_batch_steps(per_launch, b->d_insts, b->d_tiles, b->ntiles,
                                                   b->pool[b->cur], b->pool[1 - b->cur], b->off32,
                                                   mode_one_wave(c[0]), b->stream, true, true),
                           "batch multi-step launch");
                else
                    LB_HIP(lbm::launch_batch_step(b->d_insts, b->d_tiles, b->ntiles, b->tx, b->ty,
                                                  b->pool[b->cur], b->pool[1 - b->cur], b->stream,
                                                  true, true),
                           "batch step launch");
            }
            return LB_OK;
        };
        if ((st = trial(1)) != LB_OK) break;
        if (hipEventRecord(e0, b->stream) != hipSuccess) { st = fail(LB_ERR_HIP, "event"); break; }
        if ((st = trial(steps_per_trial)) != LB_OK) break;
        if (hipEventRecord(e1, b->stream) != hipSuccess) { st = fail(LB_ERR_HIP, "event"); break; }
        if (hipEventSynchronize(e1) != hipSuccess) { st = fail(LB_ERR_HIP, "event sync"); break; }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= (float)per_launch;
        if (ms < best) {
            best = ms;
            bx = c[0];
            by = c[1];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != LB_OK) return st;
    st = build_tiles(b, bx, by);
    if (st != LB_OK) return st;
    if (best_tx) *best_tx = bx;
    if (best_ty) *best_ty = by;
    return LB_OK;
}

lb_status lb_batch_macro(lb_batch* b, double* theta, double* u) {
    if (!b) return fail(LB_ERR_INVALID_ARG, "batch is NULL");
    if (!b->inited) return fail(LB_ERR_STATE, "lb_batch_macro before lb_batch_init");
    if (!theta && !u) return LB_OK;
    for (size_t i = 0; i < b->insts.size(); ++i) {
        Geo g = make_geo(&b->cfgs[i]);
        const int64_t no = b->node_offsets[i];
        LB_HIP(lbm::launch_macro(2, g, b->insts[i].r, b->pool[b->cur] + b->offsets[i],
                                 theta ? theta + no : nullptr, u ? u + 2 * no : nullptr, nullptr,
                                 b->stream),
               "batch macro launch");
    }
    return LB_OK;
}

double* lb_batch_current(const lb_batch* b) { return b ? b->pool[b->cur] : nullptr; }

}  // extern "C"
