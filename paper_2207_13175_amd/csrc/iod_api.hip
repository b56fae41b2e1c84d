// iod_api.hip -- host side of libiod: the C ABI declared in include/iod.h.
// Argument validation, the observation schedule, per-problem device tables
// (chief ephemeris and observed-angle sines/cosines) and the launch sequence
// of the particle swarm (Algorithm 1 of Zuehlke et al., AAS 22-770).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/iod.h"
#include "iod_internal.h"

using namespace iodk;

namespace {

thread_local char g_err[512];

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? IOD_ENOMEM : IOD_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

bool finite6(const double *v)
{
    for (int d = 0; d < 6; ++d)
        if (!std::isfinite(v[d])) return false;
    return true;
}

}  // namespace

struct iod_handle {
    int device = 0;
    double mu = 0, mu1 = 0, h = 0, sigma = 0, w = 0;
    int32_t K = 0, mode = 0;
    double chief[6] = {0, 0, 0, 0, 0, 0};
    std::vector<double> rc;    // [K][3] chief positions
    double *d_tab = nullptr;   // [K][TAB_W]
    int32_t *d_ns = nullptr;   // [K]

    KArgs kargs() const
    {
        KArgs A;
        A.tab = d_tab;
        A.ns = d_ns;
        A.K = K;
        A.fast = mu == 0.0 || mu >= 0x1p-60;
        A.mode = mode;
        A.mu = mu;
        A.mu1 = mu1;
        A.h = h;
        A.h2 = 0.5 * h;
        A.h6 = h / 6.0;
        A.w = w;
        return A;
    }
};

namespace {

int check_handle(iod_handle *h)
{
    if (!h) return fail(IOD_EINVAL, "null handle");
    HIP_TRY(hipSetDevice(h->device));
    return IOD_OK;
}

int check_swarm_view(const double *x, int64_t ld, int64_t m, const void *out)
{
    if (m < 0) return fail(IOD_EINVAL, "m = %lld < 0", (long long)m);
    if (ld < m || ld < 1) return fail(IOD_EINVAL, "ld = %lld must be >= max(m, 1)", (long long)ld);
    if (m > (int64_t)0x7fffffff * BS) return fail(IOD_EINVAL, "m too large");
    if (m > 0 && (!x || !out)) return fail(IOD_EINVAL, "null device pointer");
    return IOD_OK;
}

int check_pso(const iod_pso_params *p)
{
    if (!p) return fail(IOD_EINVAL, "null iod_pso_params");
    if (!std::isfinite(p->omega) || !std::isfinite(p->eta1) || !std::isfinite(p->eta2))
        return fail(IOD_EINVAL, "non-finite omega/eta1/eta2");
    if (!finite6(p->lo) || !finite6(p->hi)) return fail(IOD_EINVAL, "non-finite box");
    for (int d = 0; d < 6; ++d)
        if (p->lo[d] > p->hi[d]) return fail(IOD_EINVAL, "lo[%d] > hi[%d]", d, d);
    return IOD_OK;
}

PsoArgs pso_args(const iod_pso_params *p)
{
    PsoArgs P;
    P.omega = p->omega;
    P.eta1 = p->eta1;
    P.eta2 = p->eta2;
    P.seed = p->seed;
    P.problem = p->problem;
    for (int d = 0; d < 6; ++d) {
        P.lo[d] = p->lo[d];
        P.hi[d] = p->hi[d];
    }
    return P;
}

int check_swarm(const iod_swarm *s, bool need_init)
{
    if (!s) return fail(IOD_EINVAL, "null iod_swarm");
    if (s->m < 1) return fail(IOD_EINVAL, "swarm m = %lld < 1", (long long)s->m);
    if (s->ld < s->m) return fail(IOD_EINVAL, "swarm ld < m");
    if (s->m > (int64_t)0x7fffffff * BS) return fail(IOD_EINVAL, "m too large");
    if (!s->x || !s->v || !s->p || !s->jp || !s->cost || !s->work)
        return fail(IOD_EINVAL, "null swarm device pointer");
    if (s->hist_len < 0) return fail(IOD_EINVAL, "hist_len < 0");
    if (s->hist_len > 0 && !s->hist) return fail(IOD_EINVAL, "hist_len > 0 with null hist");
    if (need_init && s->iter < 0) return fail(IOD_ESTATE, "swarm not initialised");
    return IOD_OK;
}

SwarmArgs swarm_args(const iod_swarm *s)
{
    SwarmArgs S;
    S.x = s->x;
    S.v = s->v;
    S.p = s->p;
    S.jp = s->jp;
    S.cost = s->cost;
    S.work = s->work;
    S.hist = s->hist_len > 0 ? s->hist : nullptr;
    S.hist_len = s->hist_len;
    S.ld = s->ld;
    S.m = s->m;
    S.nslots = num_slots(s->m);
    return S;
}

}  // namespace

extern "C" {

int iod_version(void) { return 10000; }

const char *iod_last_error(void) { return g_err; }

int iod_schedule(const double *t, int32_t n_obs, double h, int64_t *nsteps, double *tau)
{
    if (!t || !nsteps || !tau) return fail(IOD_EINVAL, "null pointer");
    if (n_obs < 1 || n_obs > IOD_MAX_OBS) return fail(IOD_EINVAL, "n_obs = %d out of range", n_obs);
    if (!(h > 0.0) || !std::isfinite(h)) return fail(IOD_EINVAL, "h must be positive and finite");
    for (int32_t k = 0; k < n_obs; ++k) {
        const double tk = t[k];
        if (!std::isfinite(tk) || tk < 0.0) return fail(IOD_EINVAL, "obs_times[%d] invalid", k);
        if (k > 0 && !(tk > t[k - 1]))
            return fail(IOD_EINVAL, "obs_times not strictly increasing at %d", k);
        const double q = tk / h;
        if (q > 2147483647.0)
            return fail(IOD_EINVAL, "obs_times[%d]/h exceeds 2^31 - 1 steps", k);
        // nearest grid point, accepted within 1e-9 h
        const int64_t near = (int64_t)std::floor(q + 0.5);
        if (std::fabs(tk - (double)near * h) <= 1e-9 * h) {
            nsteps[k] = near;
            tau[k] = 0.0;
        } else {
            const int64_t below = (int64_t)std::floor(q);
            nsteps[k] = below;
            tau[k] = tk - (double)below * h;
        }
    }
    return IOD_OK;
}

int iod_create(double mu, const double chief_state[6], const double *obs_times,
               const double *obs_angles, int32_t n_obs, double sigma, const iod_options *opt,
               iod_handle **out)
{
    if (!out) return fail(IOD_EINVAL, "null out");
    *out = nullptr;
    if (!chief_state || !obs_times || !obs_angles) return fail(IOD_EINVAL, "null host pointer");
    if (!std::isfinite(mu) || mu < 0.0 || mu > 0.5) return fail(IOD_EINVAL, "mu must lie in [0, 0.5]");
    if (!finite6(chief_state)) return fail(IOD_EINVAL, "non-finite chief state");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(IOD_EINVAL, "sigma must be positive and finite");
    if (n_obs < 1 || n_obs > IOD_MAX_OBS) return fail(IOD_EINVAL, "n_obs = %d out of range", n_obs);
    iod_options o{1e-3, IOD_COST_PAPER, 0};
    if (opt) o = *opt;
    if (o.cost_mode != IOD_COST_PAPER && o.cost_mode != IOD_COST_CHI2)
        return fail(IOD_EINVAL, "unknown cost_mode %d", o.cost_mode);
    if (o.reserved != 0) return fail(IOD_EINVAL, "options.reserved must be 0");
    for (int32_t k = 0; k < 2 * n_obs; ++k)
        if (!std::isfinite(obs_angles[k])) return fail(IOD_EINVAL, "non-finite obs_angles[%d]", k);
    std::vector<int64_t> ns(n_obs);
    std::vector<double> tau(n_obs);
    int rc = iod_schedule(obs_times, n_obs, o.h, ns.data(), tau.data());
    if (rc != IOD_OK) return rc;

    iod_handle *h = new (std::nothrow) iod_handle;
    if (!h) return fail(IOD_ENOMEM, "host allocation");
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipGetDevice");
    }
    h->mu = mu;
    h->mu1 = 1.0 - mu;
    h->h = o.h;
    h->sigma = sigma;
    h->w = 1.0 / (sigma * sigma);
    h->K = n_obs;
    h->mode = o.cost_mode;
    std::memcpy(h->chief, chief_state, sizeof h->chief);
    h->rc.assign(3 * (size_t)n_obs, 0.0);

    std::vector<double> tab((size_t)n_obs * TAB_W, 0.0);
    std::vector<int32_t> ns32(n_obs);
    for (int32_t k = 0; k < n_obs; ++k) ns32[k] = (int32_t)ns[k];
    for (int32_t k = 0; k < n_obs; ++k) {
        double *row = &tab[(size_t)k * TAB_W];
        row[TAB_NS] = (double)ns[k];
        row[TAB_TAU] = tau[k];
        row[TAB_SA] = std::sin(obs_angles[2 * k]);
        row[TAB_CA] = std::cos(obs_angles[2 * k]);
        row[TAB_SB] = std::sin(obs_angles[2 * k + 1]);
        row[TAB_CB] = std::cos(obs_angles[2 * k + 1]);
    }

    // Chief ephemeris: propagate the chief with the particle propagator.
    double *d_x = nullptr, *d_st = nullptr;
    std::vector<double> st((size_t)n_obs * 6);
    auto cleanup = [&](int code) {
        if (d_x) (void)hipFree(d_x);
        if (d_st) (void)hipFree(d_st);
        if (code != IOD_OK) {
            if (h->d_tab) (void)hipFree(h->d_tab);
            if (h->d_ns) (void)hipFree(h->d_ns);
            delete h;
        }
        return code;
    };
#define CREATE_TRY(expr)                                   \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return cleanup(hip_fail(e_, #expr)); \
    } while (0)
    CREATE_TRY(hipMalloc(&h->d_tab, tab.size() * sizeof(double)));
    CREATE_TRY(hipMalloc(&h->d_ns, ns32.size() * sizeof(int32_t)));
    CREATE_TRY(hipMemcpy(h->d_ns, ns32.data(), ns32.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    CREATE_TRY(hipMalloc(&d_x, 6 * sizeof(double)));
    CREATE_TRY(hipMalloc(&d_st, st.size() * sizeof(double)));
    CREATE_TRY(hipMemcpy(h->d_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
    CREATE_TRY(hipMemcpy(d_x, chief_state, 6 * sizeof(double), hipMemcpyHostToDevice));
    CREATE_TRY(launch_propagate(h->kargs(), d_x, 1, 1, d_st, nullptr));
    CREATE_TRY(hipMemcpy(st.data(), d_st, st.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int32_t k = 0; k < n_obs; ++k)
        for (int d = 0; d < 3; ++d) {
            h->rc[3 * (size_t)k + d] = st[6 * (size_t)k + d];
            tab[(size_t)k * TAB_W + TAB_RC + d] = st[6 * (size_t)k + d];
        }
    CREATE_TRY(hipMemcpy(h->d_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
#undef CREATE_TRY
    *out = h;
    return cleanup(IOD_OK);
}

int iod_destroy(iod_handle *h)
{
    if (!h) return IOD_OK;
    int rc = IOD_OK;
    if (hipSetDevice(h->device) == hipSuccess) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) rc = hip_fail(e, "hipDeviceSynchronize");
        if (h->d_tab) {
            e = hipFree(h->d_tab);
            if (e != hipSuccess && rc == IOD_OK) rc = hip_fail(e, "hipFree");
        }
        if (h->d_ns) {
            e = hipFree(h->d_ns);
            if (e != hipSuccess && rc == IOD_OK) rc = hip_fail(e, "hipFree");
        }
    }
    delete h;
    return rc;
}

int32_t iod_num_obs(const iod_handle *h)
{
    if (!h) return fail(IOD_EINVAL, "null handle");
    return h->K;
}

int iod_chief_positions(const iod_handle *h, double *out)
{
    if (!h || !out) return fail(IOD_EINVAL, "null pointer");
    std::memcpy(out, h->rc.data(), h->rc.size() * sizeof(double));
    return IOD_OK;
}

int iod_propagate(iod_handle *h, const double *x, int64_t ld, int64_t m, double *states,
                  void *stream)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_swarm_view(x, ld, m, states);
    if (rc != IOD_OK || m == 0) return rc;
    HIP_TRY(launch_propagate(h->kargs(), x, ld, m, states, (hipStream_t)stream));
    return IOD_OK;
}

int iod_predict(iod_handle *h, const double *x, int64_t ld, int64_t m, double *angles,
                void *stream)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_swarm_view(x, ld, m, angles);
    if (rc != IOD_OK || m == 0) return rc;
    HIP_TRY(launch_predict(h->kargs(), x, ld, m, angles, (hipStream_t)stream));
    return IOD_OK;
}

int iod_eval_swarm(iod_handle *h, const double *x, int64_t ld, int64_t m, double *cost,
                   void *stream)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_swarm_view(x, ld, m, cost);
    if (rc != IOD_OK || m == 0) return rc;
    HIP_TRY(launch_eval(h->kargs(), x, ld, m, cost, (hipStream_t)stream));
    return IOD_OK;
}

int64_t iod_swarm_work_len(int64_t m)
{
    if (m < 1) return fail(IOD_EINVAL, "m = %lld < 1", (long long)m);
    return work_len(m);
}

int iod_swarm_init(iod_handle *h, iod_swarm *s, const iod_pso_params *p, void *stream)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_swarm(s, false);
    if (rc == IOD_OK) rc = check_pso(p);
    if (rc != IOD_OK) return rc;
    s->iter = -1;
    HIP_TRY(launch_swarm_init(h->kargs(), pso_args(p), swarm_args(s), (hipStream_t)stream));
    s->iter = 0;
    return IOD_OK;
}

int iod_step(iod_handle *h, iod_swarm *s, const iod_pso_params *p, int64_t n_iter, void *stream)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_swarm(s, true);
    if (rc == IOD_OK) rc = check_pso(p);
    if (rc != IOD_OK) return rc;
    if (n_iter < 0) return fail(IOD_EINVAL, "n_iter < 0");
    const KArgs A = h->kargs();
    const PsoArgs P = pso_args(p);
    const SwarmArgs S = swarm_args(s);
    for (int64_t j = 0; j < n_iter; ++j) {
        HIP_TRY(launch_swarm_iter(A, P, S, s->iter + 1, (hipStream_t)stream));
        s->iter += 1;
    }
    return IOD_OK;
}

int iod_swarm_best(iod_handle *h, iod_swarm *s, double best_state[6], double *best_cost,
                   int64_t *best_index, void *stream)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_swarm(s, true);
    if (rc != IOD_OK) return rc;
    const SwarmArgs S = swarm_args(s);
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(launch_swarm_final(S, s->iter, st));
    double rec[REC];
    const double *d_rec = s->work + 2 * S.nslots * REC + (s->iter & 1) * REC;
    HIP_TRY(hipMemcpyAsync(rec, d_rec, sizeof rec, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (best_state) std::memcpy(best_state, rec + 2, 6 * sizeof(double));
    if (best_cost) *best_cost = rec[0];
    if (best_index) *best_index = (int64_t)rec[1];
    return IOD_OK;
}

int iod_solve(iod_handle *h, const iod_pso_params *p, int64_t m, int64_t n_iter,
              double best_state[6], double *best_cost, double *history)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_pso(p);
    if (rc != IOD_OK) return rc;
    if (m < 1 || m > (int64_t)0x7fffffff * BS) return fail(IOD_EINVAL, "m out of range");
    if (n_iter < 0) return fail(IOD_EINVAL, "n_iter < 0");
    const int64_t ld = (m + 63) / 64 * 64;
    const int64_t wl = work_len(m);
    const size_t total = (size_t)(20 * ld + wl + (n_iter + 1));
    double *buf = nullptr;
    hipStream_t st = nullptr;
    HIP_TRY(hipStreamCreate(&st));
    hipError_t e = hipMalloc(&buf, total * sizeof(double));
    if (e != hipSuccess) {
        (void)hipStreamDestroy(st);
        return hip_fail(e, "hipMalloc");
    }
    iod_swarm s;
    s.x = buf;
    s.v = buf + 6 * ld;
    s.p = buf + 12 * ld;
    s.jp = buf + 18 * ld;
    s.cost = buf + 19 * ld;
    s.work = buf + 20 * ld;
    s.hist = buf + 20 * ld + wl;
    s.hist_len = n_iter + 1;
    s.ld = ld;
    s.m = m;
    s.iter = -1;
    rc = iod_swarm_init(h, &s, p, st);
    if (rc == IOD_OK) rc = iod_step(h, &s, p, n_iter, st);
    if (rc == IOD_OK) rc = iod_swarm_best(h, &s, best_state, best_cost, nullptr, st);
    if (rc == IOD_OK && history) {
        e = hipMemcpy(history, s.hist, (size_t)(n_iter + 1) * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = hip_fail(e, "hipMemcpy history");
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    (void)hipStreamDestroy(st);
    return rc;
}

}  // extern "C"
