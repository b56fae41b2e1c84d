// iod_api.hip -- host side of libiod: the C ABI declared in include/iod.h.
// Argument validation, the observation schedule, per-problem device tables
// (chief ephemeris and observed-angle sines/cosines), work lists and the
// launch sequence of the particle swarm (Algorithm 1 of Zuehlke et al.,
// AAS 22-770), for one problem or a batch of independent problems.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/iod.h"
#include "iod_launch.h"

using namespace iodk;

namespace {

// A named range around a host-side phase, for tools that record markers
// (rocprofv3 --marker-trace); a no-op call when none is attached. Phases that
// enqueue device work end after synchronising their stream, so the range
// covers the device time.
class Phase {
public:
    explicit Phase(const char *name) { roctxRangePush(name); }
    void end()
    {
        if (open_) roctxRangePop();
        open_ = false;
    }
    ~Phase() { end(); }
    Phase(const Phase &) = delete;
    Phase &operator=(const Phase &) = delete;

private:
    bool open_ = true;
};

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

#define HIP_TRY(expr)                                     \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

bool finite6(const double *v)
{
    for (int d = 0; d < 6; ++d)
        if (!std::isfinite(v[d])) return false;
    return true;
}

constexpr int64_t MAX_M = (int64_t)1 << 40;
constexpr int DEFAULT_BLOCK = 256;

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
int64_t round64(int64_t a) { return ceil_div(a, 64) * 64; }

// Host-side description of one problem, validated, with its observation
// table rows (chief positions filled in on the device).
struct HostProblem {
    double mu = 0, h = 0, sigma = 0;
    double sigma_range = 0;     // > 0: range measurements in TAB_RANGE
    int32_t K = 0, mode = 0;
    double chief[6] = {0, 0, 0, 0, 0, 0};
    std::vector<double> tab;    // [K][TAB_W]
    std::vector<int32_t> ns;    // [K]
    int64_t steps = 0;          // RK4 steps of one evaluation
};

int check_config(const iod_launch_config *c)
{
    if (!c) return fail(IOD_EINVAL, "null iod_launch_config");
    if (c->block != 0 && c->block != 64 && c->block != 128 && c->block != 256)
        return fail(IOD_EINVAL, "block must be 0, 64, 128 or 256");
    if (c->order != IOD_ORDER_LONGEST_FIRST && c->order != IOD_ORDER_PROBLEM)
        return fail(IOD_EINVAL, "unknown order %d", c->order);
    if (c->graph != 0 && c->graph != 1) return fail(IOD_EINVAL, "graph must be 0 or 1");
    if (c->waves != 0 && c->waves != 3) return fail(IOD_EINVAL, "waves must be 0 or 3");
    return IOD_OK;
}

int block_of(const iod_launch_config &c) { return c.block ? c.block : DEFAULT_BLOCK; }

}  // namespace

extern "C" int iod_schedule(const double *t, int32_t n_obs, double h, int64_t *nsteps, double *tau);

namespace {

int make_problem(double mu, const double *chief, const double *t, const double *ang,
                 const double *ranges, int32_t K, double sigma, double sigma_range,
                 const iod_options *opt, HostProblem &P)
{
    if (!chief || !t || !ang) return fail(IOD_EINVAL, "null host pointer");
    if (ranges) {
        if (!(sigma_range > 0.0) || !std::isfinite(sigma_range))
            return fail(IOD_EINVAL, "sigma_range must be positive and finite");
        for (int32_t k = 0; k < K; ++k)
            if (!std::isfinite(ranges[k]) || ranges[k] < 0.0)
                return fail(IOD_EINVAL, "obs_ranges[%d] invalid", k);
    }
    if (!std::isfinite(mu) || mu < 0.0 || mu > 0.5) return fail(IOD_EINVAL, "mu must lie in [0, 0.5]");
    if (!finite6(chief)) return fail(IOD_EINVAL, "non-finite chief state");
    if (!(sigma > 0.0) || !std::isfinite(sigma))
        return fail(IOD_EINVAL, "sigma must be positive and finite");
    if (K < 1 || K > IOD_MAX_OBS) return fail(IOD_EINVAL, "n_obs = %d out of range", K);
    iod_options o{1e-3, IOD_COST_PAPER, 0};
    if (opt) o = *opt;
    if (o.cost_mode != IOD_COST_PAPER && o.cost_mode != IOD_COST_CHI2)
        return fail(IOD_EINVAL, "unknown cost_mode %d", o.cost_mode);
    if (o.reserved != 0) return fail(IOD_EINVAL, "options.reserved must be 0");
    for (int32_t k = 0; k < 2 * K; ++k)
        if (!std::isfinite(ang[k])) return fail(IOD_EINVAL, "non-finite obs_angles[%d]", k);
    std::vector<int64_t> ns(K);
    std::vector<double> tau(K);
    int rc = iod_schedule(t, K, o.h, ns.data(), tau.data());
    if (rc != IOD_OK) return rc;
    P.mu = mu;
    P.h = o.h;
    P.sigma = sigma;
    P.sigma_range = ranges ? sigma_range : 0.0;
    P.K = K;
    P.mode = o.cost_mode;
    std::memcpy(P.chief, chief, sizeof P.chief);
    P.tab.assign((size_t)K * TAB_W, 0.0);
    P.ns.resize(K);
    for (int32_t k = 0; k < K; ++k) {
        double *row = &P.tab[(size_t)k * TAB_W];
        P.ns[k] = (int32_t)ns[k];
        row[TAB_NS] = (double)ns[k];
        row[TAB_TAU] = tau[k];
        row[TAB_SA] = std::sin(ang[2 * k]);
        row[TAB_CA] = std::cos(ang[2 * k]);
        row[TAB_SB] = std::sin(ang[2 * k + 1]);
        row[TAB_CB] = std::cos(ang[2 * k + 1]);
        row[TAB_RANGE] = ranges ? ranges[k] : 0.0;
    }
    P.steps = ns[K - 1] + (tau[K - 1] != 0.0 ? 1 : 0);
    return IOD_OK;
}

// Chief data of the FP32 propagation of one problem, in the tables of its
// handle or batch (null until built).
struct ChiefTables {
    const float *cst = nullptr, *cpt = nullptr;
    const double *cobs = nullptr;
};

// Sizes of a problem's chief tables: floats of the per-step rows (padded by
// CST_CHUNK steps), floats of the per-observation partial-step rows, doubles
// of the states at t = 0 and at the observations.
int64_t cst_floats(const HostProblem &P) { return ((int64_t)P.ns[P.K - 1] + CST_CHUNK) * CST_STEP; }
int64_t cpt_floats(const HostProblem &P) { return (int64_t)P.K * CST_STEP; }
int64_t cobs_doubles(const HostProblem &P) { return ((int64_t)P.K + 1) * 6; }

KArgs kargs_of(const HostProblem &P, const double *d_tab, const int32_t *d_ns,
               const ChiefTables &T = ChiefTables())
{
    KArgs A;
    A.cst = T.cst;
    A.cpt = T.cpt;
    A.cobs = T.cobs;
    A.tab = d_tab;
    A.ns = d_ns;
    A.K = P.K;
    A.mode = P.mode;
    A.fast = true;   // the in-range sequences hold for every mu (see rhs)
    A.mu = P.mu;
    A.mu1 = 1.0 - P.mu;
    A.h = P.h;
    A.h2 = 0.5 * P.h;
    A.h6 = P.h / 6.0;
    A.w = 1.0 / (P.sigma * P.sigma);
    A.wr = P.sigma_range > 0.0 ? 1.0 / (P.sigma_range * P.sigma_range) : 0.0;
    return A;
}

// Levels per dimension of the grid initialisation for m particles: b levels
// everywhere with b^6 <= m < (b+1)^6, then dimensions 0, 1, ... raised to
// b + 1 while the product stays <= m. Returns the product.
int64_t grid_levels(int64_t m, int64_t n[6])
{
    int64_t b = 1;
    while (true) {
        const int64_t c = b + 1;
        int64_t pw = 1;
        for (int d = 0; d < 6; ++d) pw *= c;
        if (pw > m) break;
        b = c;
    }
    int64_t g = 1;
    for (int d = 0; d < 6; ++d) {
        n[d] = b;
        g *= b;
    }
    for (int d = 0; d < 6 && g / b * (b + 1) <= m; ++d) {
        g = g / b * (b + 1);
        n[d] = b + 1;
    }
    return g;
}

// Constriction factor for phi = eta1 + eta2 > 4 (eq. constriction:factor).
double constriction(double eta1, double eta2)
{
    const double phi = eta1 + eta2;
    return 2.0 / std::fabs(2.0 - phi - std::sqrt(phi * phi - 4.0 * phi));
}

ProbDesc desc_of(const KArgs &A, const double chief[6], const iod_pso_params *p)
{
    ProbDesc D;
    std::memset(&D, 0, sizeof D);
    D.k = A;
    std::memcpy(D.chief, chief, sizeof D.chief);
    D.kappa = 1.0;
    if (p) {
        D.omega = p->omega;
        D.eta1 = p->eta1;
        D.eta2 = p->eta2;
        std::memcpy(D.lo, p->lo, sizeof D.lo);
        std::memcpy(D.hi, p->hi, sizeof D.hi);
        D.seed = p->seed;
        D.problem = p->problem;
        D.flags = p->flags & PSO_PER_DIM_R;
        if (p->flags & IOD_PSO_CONSTRICTION) D.kappa = constriction(p->eta1, p->eta2);
        D.tol = p->tol;
        D.tol_lag = p->tol > 0.0 ? p->tol_lag : 0;
    }
    return D;
}

// Grid levels of a swarm of m particles, when the initialisation asks for it.
void set_grid(ProbDesc &D, const iod_pso_params *p, int64_t m)
{
    D.grid_g = 0;
    if (p && (p->flags & IOD_PSO_GRID_INIT) && m >= 1) D.grid_g = grid_levels(m, D.grid_n);
}

int check_pso(const iod_pso_params *p)
{
    if (!p) return fail(IOD_EINVAL, "null iod_pso_params");
    if (!std::isfinite(p->omega) || !std::isfinite(p->eta1) || !std::isfinite(p->eta2))
        return fail(IOD_EINVAL, "non-finite omega/eta1/eta2");
    if (!finite6(p->lo) || !finite6(p->hi)) return fail(IOD_EINVAL, "non-finite box");
    for (int d = 0; d < 6; ++d)
        if (p->lo[d] > p->hi[d]) return fail(IOD_EINVAL, "lo[%d] > hi[%d]", d, d);
    const uint32_t known = IOD_PSO_CONSTRICTION | IOD_PSO_PER_DIM_R | IOD_PSO_GRID_INIT;
    if (p->flags & ~known) return fail(IOD_EINVAL, "unknown flags 0x%x", p->flags & ~known);
    if ((p->flags & IOD_PSO_CONSTRICTION) && !(p->eta1 + p->eta2 > 4.0))
        return fail(IOD_EINVAL, "constriction factor needs eta1 + eta2 > 4");
    if (!std::isfinite(p->tol) || p->tol < 0.0) return fail(IOD_EINVAL, "tol must be finite and >= 0");
    if (p->tol > 0.0 && p->tol_lag < 1) return fail(IOD_EINVAL, "tol_lag must be >= 1");
    return IOD_OK;
}

// RAII device buffers for the synchronous entry points.
struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

// Device buffer kept by a handle or batch across calls and grown on demand,
// so that a repeated call of the same or a smaller size allocates nothing.
// Growing frees the old buffer first (hipFree waits for the device).
struct DevCache {
    void *p = nullptr;
    size_t bytes = 0;
    DevCache() = default;
    DevCache(const DevCache &) = delete;
    DevCache &operator=(const DevCache &) = delete;
    ~DevCache() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t n)
    {
        if (n == 0) n = 1;
        if (n <= bytes) return hipSuccess;
        release();
        Phase ph("libiod: device allocation");
        hipError_t e = hipMalloc(&p, n);
        if (e == hipSuccess)
            bytes = n;
        else
            p = nullptr;
        return e;
    }
    template <class T>
    T *as() const
    {
        return (T *)p;
    }
};

// Device copy of a host table, copied (stream-ordered, from pageable host
// memory, which the runtime stages before returning) only when its bytes
// differ from the last copy; the last copy's bytes are kept as the shadow.
// A table that kernels modify must not use this (its device bytes would no
// longer match the shadow).
struct DevTable {
    DevCache d;
    std::vector<unsigned char> shadow;
    bool valid = false;
    hipError_t upload(const void *src, size_t n, hipStream_t st)
    {
        if (valid && shadow.size() == n && (n == 0 || std::memcmp(shadow.data(), src, n) == 0))
            return hipSuccess;
        valid = false;
        hipError_t e = d.ensure(n);
        if (e != hipSuccess) return e;
        shadow.assign((const unsigned char *)src, (const unsigned char *)src + n);
        if (n) e = hipMemcpyAsync(d.p, shadow.data(), n, hipMemcpyHostToDevice, st);
        valid = e == hipSuccess;
        return e;
    }
    template <class T>
    hipError_t upload(const std::vector<T> &v, hipStream_t st)
    {
        return upload(v.data(), v.size() * sizeof(T), st);
    }
    template <class T>
    T *as() const
    {
        return d.as<T>();
    }
};

// Bytes that identify a captured launch sequence: everything its kernel
// arguments were built from.
struct Key {
    std::vector<unsigned char> b;
    template <class T>
    Key &add(const T &v)
    {
        const unsigned char *q = (const unsigned char *)&v;
        b.insert(b.end(), q, q + sizeof v);
        return *this;
    }
};

// Instantiated graphs of iteration sequences, keyed by their launch
// arguments, most recently used last; at most MAX are kept.
struct GraphCache {
    static constexpr size_t MAX = 32;
    struct Entry {
        std::vector<unsigned char> key;
        hipGraphExec_t exec;
    };
    std::vector<Entry> entries;
    GraphCache() = default;
    GraphCache(const GraphCache &) = delete;
    GraphCache &operator=(const GraphCache &) = delete;
    ~GraphCache() { clear(); }
    void clear()
    {
        for (Entry &e : entries)
            if (e.exec) (void)hipGraphExecDestroy(e.exec);
        entries.clear();
    }
    hipGraphExec_t find(const Key &k)
    {
        for (size_t i = 0; i < entries.size(); ++i)
            if (entries[i].key == k.b) {
                Entry e = entries[i];
                entries.erase(entries.begin() + (long)i);
                entries.push_back(e);
                return e.exec;
            }
        return nullptr;
    }
    void put(const Key &k, hipGraphExec_t exec)
    {
        if (entries.size() >= MAX) {
            (void)hipGraphExecDestroy(entries.front().exec);
            entries.erase(entries.begin());
        }
        entries.push_back({k.b, exec});
    }
};

// Runs the iteration launches n0 + 1 .. n0 + n_iter, directly or as one
// captured graph. With a cache, the graph is instantiated once per key
// (which must identify every launch argument) and replayed afterwards.
template <class F>
int run_iterations(hipStream_t st, bool graph, int64_t n0, int64_t n_iter, F launch_one,
                   GraphCache *cache = nullptr, Key key = Key())
{
    if (!graph || n_iter == 0) {
        for (int64_t j = 1; j <= n_iter; ++j) HIP_TRY(launch_one(n0 + j));
        return IOD_OK;
    }
    key.add(n0).add(n_iter);
    if (cache) {
        if (hipGraphExec_t ex = cache->find(key)) {
            HIP_TRY(hipGraphLaunch(ex, st));
            return IOD_OK;
        }
    }
    Phase ph("libiod: graph capture and instantiation");
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    for (int64_t j = 1; j <= n_iter && le == hipSuccess; ++j) le = launch_one(n0 + j);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(st, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le, "iteration launch under capture");
    }
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    hipGraphExec_t ge = nullptr;
    hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    ph.end();
    if (e == hipSuccess) e = hipGraphLaunch(ge, st);
    if (e != hipSuccess) {
        if (ge) (void)hipGraphExecDestroy(ge);
        return hip_fail(e, "hipGraph instantiate/launch");
    }
    if (cache)
        cache->put(key, ge);
    else
        (void)hipGraphExecDestroy(ge);
    return IOD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Single problem
// ---------------------------------------------------------------------------

struct iod_handle {
    int device = 0;
    HostProblem P;
    double *d_tab = nullptr;   // [K][TAB_W]
    int32_t *d_ns = nullptr;   // [K]
    std::vector<double> rc;    // [K][3] chief positions
    iod_launch_config cfg{0, IOD_ORDER_LONGEST_FIRST, 0, 0};
    // kept across iod_solve calls: its stream, swarm storage and graphs
    hipStream_t stream = nullptr;
    DevCache solve_buf;
    GraphCache graphs;
    // FP32 formulation, and the chief data of the offset formulation, built
    // on its first call
    int32_t fp32_mode = IOD_FP32_RELATIVE;
    DevCache cst, cpt, cobs;
    bool chief_built = false;

    KArgs kargs() const
    {
        ChiefTables T;
        if (chief_built) {
            T.cst = cst.as<const float>();
            T.cpt = cpt.as<const float>();
            T.cobs = cobs.as<const double>();
        }
        return kargs_of(P, d_tab, d_ns, T);
    }
};

// Buffers of the batched refinement stage, kept across calls.
struct PolishBuffers {
    DevCache cand, x, chi, work, best, bchi, cost, act, done, vt, jrows, live, live_count;
    DevTable desc, edesc, tdesc, list, lanes, nn;
};

struct iod_batch {
    int device = 0;
    int32_t P = 0;
    std::vector<HostProblem> probs;
    std::vector<int64_t> tab_off;  // per problem, rows
    double *d_tab = nullptr;       // concatenated [sum K][TAB_W]
    int32_t *d_ns = nullptr;       // concatenated [sum K]
    iod_launch_config cfg{0, IOD_ORDER_LONGEST_FIRST, 1, 0};
    double last_iter_ms = 0.0;  // mean iteration time of the last iod_batch_solve
    // kept across calls, so that repeated solves of one shape allocate and
    // instantiate nothing: the solve stream and timing events, the swarm
    // storage, the launch tables, the captured iteration graphs, and the
    // tables of the evaluation, selection and polish calls
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    DevCache swarm, cand;
    DevTable desc, work, porder;
    GraphCache graphs;
    DevTable eval_desc, eval_work, topk_desc, bpol_desc, bpol_work;
    PolishBuffers pol;
    // FP32 formulation, and the chief data of the offset formulation, built
    // on its first call: per-problem offsets into the three tables
    int32_t fp32_mode = IOD_FP32_RELATIVE;
    DevCache cst, cpt, cobs;
    std::vector<int64_t> cst_off, cpt_off, cobs_off;
    bool chief_built = false;

    KArgs kargs(int32_t p) const
    {
        ChiefTables T;
        if (chief_built) {
            T.cst = cst.as<const float>() + cst_off[p];
            T.cpt = cpt.as<const float>() + cpt_off[p];
            T.cobs = cobs.as<const double>() + cobs_off[p];
        }
        return kargs_of(probs[p], d_tab + tab_off[p] * TAB_W, d_ns + tab_off[p], T);
    }
};

namespace {

int check_handle(iod_handle *h)
{
    if (!h) return fail(IOD_EINVAL, "null handle");
    HIP_TRY(hipSetDevice(h->device));
    return IOD_OK;
}

int check_batch(iod_batch *b)
{
    if (!b) return fail(IOD_EINVAL, "null batch");
    HIP_TRY(hipSetDevice(b->device));
    return IOD_OK;
}

// Build the chief data of the FP32 propagation (once per handle or batch):
// allocate the three tables, then one thread per problem propagates its
// chief in FP64 and fills them. Synchronous.
int build_chief_tables(const std::vector<ProbDesc> &descs)
{
    DevBuf d;
    HIP_TRY(hipMalloc(&d.p, descs.size() * sizeof(ProbDesc)));
    HIP_TRY(hipMemcpy(d.p, descs.data(), descs.size() * sizeof(ProbDesc), hipMemcpyHostToDevice));
    HIP_TRY(launch_chief_stages((const ProbDesc *)d.p, (int64_t)descs.size(), nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return IOD_OK;
}

int ensure_chief_tables(iod_handle *h)
{
    if (h->chief_built) return IOD_OK;
    Phase ph("libiod: chief tables of the FP32 propagation");
    HIP_TRY(h->cst.ensure((size_t)cst_floats(h->P) * sizeof(float)));
    HIP_TRY(h->cpt.ensure((size_t)cpt_floats(h->P) * sizeof(float)));
    HIP_TRY(h->cobs.ensure((size_t)cobs_doubles(h->P) * sizeof(double)));
    h->chief_built = true;
    int rc = build_chief_tables({desc_of(h->kargs(), h->P.chief, nullptr)});
    if (rc != IOD_OK) h->chief_built = false;
    return rc;
}

int ensure_chief_tables(iod_batch *b)
{
    if (b->chief_built) return IOD_OK;
    Phase ph("libiod: chief tables of the FP32 propagation");
    b->cst_off.assign(b->P, 0);
    b->cpt_off.assign(b->P, 0);
    b->cobs_off.assign(b->P, 0);
    int64_t ncst = 0, ncpt = 0, ncobs = 0;
    for (int32_t p = 0; p < b->P; ++p) {
        b->cst_off[p] = ncst;
        b->cpt_off[p] = ncpt;
        b->cobs_off[p] = ncobs;
        ncst += cst_floats(b->probs[p]);
        ncpt += cpt_floats(b->probs[p]);
        ncobs += cobs_doubles(b->probs[p]);
    }
    HIP_TRY(b->cst.ensure((size_t)ncst * sizeof(float)));
    HIP_TRY(b->cpt.ensure((size_t)ncpt * sizeof(float)));
    HIP_TRY(b->cobs.ensure((size_t)ncobs * sizeof(double)));
    b->chief_built = true;
    std::vector<ProbDesc> descs(b->P);
    for (int32_t p = 0; p < b->P; ++p) descs[p] = desc_of(b->kargs(p), b->probs[p].chief, nullptr);
    int rc = build_chief_tables(descs);
    if (rc != IOD_OK) b->chief_built = false;
    return rc;
}

int check_swarm_view(const double *x, int64_t ld, int64_t m, const void *out)
{
    if (m < 0) return fail(IOD_EINVAL, "m = %lld < 0", (long long)m);
    if (ld < m || ld < 1) return fail(IOD_EINVAL, "ld = %lld must be >= max(m, 1)", (long long)ld);
    if (m > MAX_M) return fail(IOD_EINVAL, "m too large");
    if (m > 0 && (!x || !out)) return fail(IOD_EINVAL, "null device pointer");
    return IOD_OK;
}

int check_swarm(const iod_swarm *s, bool need_init)
{
    if (!s) return fail(IOD_EINVAL, "null iod_swarm");
    if (s->m < 1) return fail(IOD_EINVAL, "swarm m = %lld < 1", (long long)s->m);
    if (s->ld < s->m) return fail(IOD_EINVAL, "swarm ld < m");
    if (s->m > MAX_M) return fail(IOD_EINVAL, "m too large");
    if (!s->x || !s->v || !s->p || !s->jp || !s->cost || !s->work)
        return fail(IOD_EINVAL, "null swarm device pointer");
    if (s->hist_len < 0) return fail(IOD_EINVAL, "hist_len < 0");
    if (s->hist_len > 0 && !s->hist) return fail(IOD_EINVAL, "hist_len > 0 with null hist");
    if (need_init) {
        if (s->iter < 0) return fail(IOD_ESTATE, "swarm not initialised");
        if (s->block != 64 && s->block != 128 && s->block != 256)
            return fail(IOD_ESTATE, "swarm block %d invalid (not initialised?)", s->block);
    }
    return IOD_OK;
}

// Launch view of a caller-owned single-problem swarm.
void single_view(const iod_handle *h, const iod_swarm *s, const iod_pso_params *p, ProbDesc &D,
                 SwarmArrays &B)
{
    const int64_t nslots = ceil_div(s->m, s->block);
    D = desc_of(h->kargs(), h->P.chief, p);
    D.hist = s->hist_len > 0 ? s->hist : nullptr;
    D.hist_len = s->hist_len;
    D.m = s->m;
    D.off = 0;
    D.slot_off = 0;
    D.nslots = nslots;
    D.block = s->block;
    B.desc = nullptr;
    B.work = nullptr;
    B.x = s->x;
    B.v = s->v;
    B.p = s->p;
    B.jp = s->jp;
    B.cost = s->cost;
    B.slots = s->work;
    B.recs = s->work + 2 * nslots * REC;
    B.stop = B.recs + 2 * REC;
    B.porder = nullptr;
    set_grid(D, p, s->m);
    B.ld = s->ld;
    B.total_slots = nslots;
    B.nprob = 1;
}

}  // namespace

extern "C" {

int iod_version(void) { return 10200; }

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
        if (q > 2147483646.0)
            return fail(IOD_EINVAL, "obs_times[%d]/h exceeds 2^31 - 2 steps", k);
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
    return iod_create_ranged(mu, chief_state, obs_times, obs_angles, nullptr, n_obs, sigma, 0.0,
                             opt, out);
}

int iod_create_ranged(double mu, const double chief_state[6], const double *obs_times,
                      const double *obs_angles, const double *obs_ranges, int32_t n_obs,
                      double sigma, double sigma_range, const iod_options *opt,
                      iod_handle **out)
{
    if (!out) return fail(IOD_EINVAL, "null out");
    *out = nullptr;
    HostProblem P;
    int rc = make_problem(mu, chief_state, obs_times, obs_angles, obs_ranges, n_obs, sigma,
                          sigma_range, opt, P);
    if (rc != IOD_OK) return rc;
    iod_handle *h = new (std::nothrow) iod_handle;
    if (!h) return fail(IOD_ENOMEM, "host allocation");
    h->P = std::move(P);
    auto bail = [&](int code) {
        iod_destroy(h);
        return code;
    };
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) return bail(hip_fail(e, "hipGetDevice"));
    const size_t K = (size_t)h->P.K;
    if ((e = hipMalloc(&h->d_tab, K * TAB_W * sizeof(double))) != hipSuccess)
        return bail(hip_fail(e, "hipMalloc table"));
    if ((e = hipMalloc(&h->d_ns, K * sizeof(int32_t))) != hipSuccess)
        return bail(hip_fail(e, "hipMalloc steps"));
    if ((e = hipMemcpy(h->d_tab, h->P.tab.data(), K * TAB_W * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(h->d_ns, h->P.ns.data(), K * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(hip_fail(e, "hipMemcpy tables"));
    // chief ephemeris, written into the device table
    const ProbDesc D = desc_of(h->kargs(), h->P.chief, nullptr);
    if ((e = launch_chief(D, nullptr, 1, nullptr)) != hipSuccess) return bail(hip_fail(e, "chief launch"));
    std::vector<double> tab(K * TAB_W);
    if ((e = hipMemcpy(tab.data(), h->d_tab, tab.size() * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
        return bail(hip_fail(e, "hipMemcpy chief"));
    h->rc.resize(3 * K);
    for (size_t k = 0; k < K; ++k)
        for (int d = 0; d < 3; ++d) h->rc[3 * k + d] = tab[k * TAB_W + TAB_RC + d];
    *out = h;
    return IOD_OK;
}

int iod_destroy(iod_handle *h)
{
    if (!h) return IOD_OK;
    int rc = IOD_OK;
    if (hipSetDevice(h->device) == hipSuccess) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) rc = hip_fail(e, "hipDeviceSynchronize");
        h->graphs.clear();
        h->solve_buf.release();
        if (h->stream) (void)hipStreamDestroy(h->stream);
        h->stream = nullptr;
        if (h->d_tab && (e = hipFree(h->d_tab)) != hipSuccess && rc == IOD_OK) rc = hip_fail(e, "hipFree");
        if (h->d_ns && (e = hipFree(h->d_ns)) != hipSuccess && rc == IOD_OK) rc = hip_fail(e, "hipFree");
    }
    delete h;
    return rc;
}

int iod_set_config(iod_handle *h, const iod_launch_config *cfg)
{
    if (!h) return fail(IOD_EINVAL, "null handle");
    int rc = check_config(cfg);
    if (rc != IOD_OK) return rc;
    h->cfg = *cfg;
    return IOD_OK;
}

int iod_get_config(const iod_handle *h, iod_launch_config *cfg)
{
    if (!h || !cfg) return fail(IOD_EINVAL, "null pointer");
    *cfg = h->cfg;
    return IOD_OK;
}

int iod_set_fp32_mode(iod_handle *h, int32_t mode)
{
    if (!h) return fail(IOD_EINVAL, "null handle");
    if (mode != IOD_FP32_RELATIVE && mode != IOD_FP32_ABSOLUTE)
        return fail(IOD_EINVAL, "unknown FP32 mode %d", mode);
    h->fp32_mode = mode;
    return IOD_OK;
}

int32_t iod_num_obs(const iod_handle *h)
{
    if (!h) return fail(IOD_EINVAL, "null handle");
    return h->P.K;
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

int iod_predict_ranges(iod_handle *h, const double *x, int64_t ld, int64_t m, double *ranges,
                       void *stream)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_swarm_view(x, ld, m, ranges);
    if (rc != IOD_OK || m == 0) return rc;
    HIP_TRY(launch_predict_ranges(h->kargs(), x, ld, m, ranges, (hipStream_t)stream));
    return IOD_OK;
}

int iod_eval_swarm(iod_handle *h, const double *x, int64_t ld, int64_t m, double *cost,
                   void *stream)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_swarm_view(x, ld, m, cost);
    if (rc != IOD_OK || m == 0) return rc;
    const int bs = block_of(h->cfg);
    ProbDesc D = desc_of(h->kargs(), h->P.chief, nullptr);
    D.m = m;
    D.nslots = ceil_div(m, bs);
    D.block = bs;
    SwarmArrays B;
    std::memset(&B, 0, sizeof B);
    B.x = const_cast<double *>(x);
    B.cost = cost;
    B.ld = ld;
    B.nprob = 1;
    HIP_TRY(launch_eval(D, B, bs, D.nslots, (hipStream_t)stream));
    return IOD_OK;
}

int64_t iod_swarm_work_len(int64_t m)
{
    if (m < 1 || m > MAX_M) return fail(IOD_EINVAL, "m = %lld out of range", (long long)m);
    return 2 * ceil_div(m, 64) * REC + 3 * REC;
}

int iod_swarm_init(iod_handle *h, iod_swarm *s, const iod_pso_params *p, void *stream)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_swarm(s, false);
    if (rc == IOD_OK) rc = check_pso(p);
    if (rc != IOD_OK) return rc;
    s->iter = -1;
    s->block = block_of(h->cfg);
    ProbDesc D;
    SwarmArrays B;
    single_view(h, s, p, D, B);
    HIP_TRY(launch_swarm_init(D, B, s->block, D.nslots, (hipStream_t)stream));
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
    if (p->tol > 0.0 && (!s->hist || s->hist_len < s->iter + n_iter + 1))
        return fail(IOD_EINVAL, "Algorithm 2 (tol > 0) needs a history of >= %lld entries",
                    (long long)(s->iter + n_iter + 1));
    ProbDesc D;
    SwarmArrays B;
    single_view(h, s, p, D, B);
    for (int64_t j = 1; j <= n_iter; ++j) {
        HIP_TRY(launch_swarm_iter(D, B, s->block, D.nslots, s->iter + 1, (hipStream_t)stream,
                                  h->cfg.waves));
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
    ProbDesc D;
    SwarmArrays B;
    single_view(h, s, nullptr, D, B);
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(launch_swarm_final(D, B, s->iter, st));
    double rec[REC];
    HIP_TRY(hipMemcpyAsync(rec, B.recs + (s->iter & 1) * REC, sizeof rec, hipMemcpyDeviceToHost, st));
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
    if (m < 1 || m > MAX_M) return fail(IOD_EINVAL, "m out of range");
    if (n_iter < 0) return fail(IOD_EINVAL, "n_iter < 0");
    Phase phase("iod_solve");
    const int64_t ld = round64(m);
    const int64_t wl = iod_swarm_work_len(m);
    const size_t total = (size_t)(20 * ld + wl + (n_iter + 1));
    // the stream, the swarm storage and the captured iterations are the
    // handle's, kept for the next call
    if (!h->stream) HIP_TRY(hipStreamCreate(&h->stream));
    HIP_TRY(h->solve_buf.ensure(total * sizeof(double)));
    hipStream_t st = h->stream;
    double *base = h->solve_buf.as<double>();
    iod_swarm s;
    std::memset(&s, 0, sizeof s);
    s.x = base;
    s.v = base + 6 * ld;
    s.p = base + 12 * ld;
    s.jp = base + 18 * ld;
    s.cost = base + 19 * ld;
    s.work = base + 20 * ld;
    s.hist = base + 20 * ld + wl;
    s.hist_len = n_iter + 1;
    s.ld = ld;
    s.m = m;
    s.iter = -1;
    rc = iod_swarm_init(h, &s, p, st);
    if (rc == IOD_OK) {
        ProbDesc D;
        SwarmArrays B;
        single_view(h, &s, p, D, B);
        Key key;
        key.add(D).add(B).add(s.block).add(h->cfg.waves);
        rc = run_iterations(st, h->cfg.graph != 0, 0, n_iter, [&](int64_t n) {
            return launch_swarm_iter(D, B, s.block, D.nslots, n, st, h->cfg.waves);
        }, &h->graphs, key);
        if (rc == IOD_OK) s.iter = n_iter;
    }
    if (rc == IOD_OK) rc = iod_swarm_best(h, &s, best_state, best_cost, nullptr, st);
    if (rc == IOD_OK && history) {
        hipError_t e = hipMemcpyAsync(history, s.hist, (size_t)(n_iter + 1) * sizeof(double),
                                      hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = hip_fail(e, "hipMemcpy history");
    }
    (void)hipStreamSynchronize(st);
    return rc;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------

int iod_create_batch(int32_t n_problems, const double *mu, const double *chief_states,
                     const int64_t *obs_offsets, const double *obs_times,
                     const double *obs_angles, const double *sigma, const iod_options *opt,
                     iod_batch **out)
{
    return iod_create_batch_ranged(n_problems, mu, chief_states, obs_offsets, obs_times,
                                   obs_angles, nullptr, sigma, nullptr, opt, out);
}

int iod_create_batch_ranged(int32_t n_problems, const double *mu, const double *chief_states,
                            const int64_t *obs_offsets, const double *obs_times,
                            const double *obs_angles, const double *obs_ranges,
                            const double *sigma, const double *sigma_range,
                            const iod_options *opt, iod_batch **out)
{
    if (!out) return fail(IOD_EINVAL, "null out");
    *out = nullptr;
    if (n_problems < 1) return fail(IOD_EINVAL, "n_problems = %d < 1", n_problems);
    if (!mu || !chief_states || !obs_offsets || !obs_times || !obs_angles || !sigma)
        return fail(IOD_EINVAL, "null host pointer");
    if (obs_ranges && !sigma_range) return fail(IOD_EINVAL, "obs_ranges given without sigma_range");
    if (obs_offsets[0] != 0) return fail(IOD_EINVAL, "obs_offsets[0] must be 0");
    iod_batch *b = new (std::nothrow) iod_batch;
    if (!b) return fail(IOD_ENOMEM, "host allocation");
    auto bail = [&](int code) {
        iod_batch_destroy(b);
        return code;
    };
    b->P = n_problems;
    b->probs.resize(n_problems);
    b->tab_off.resize(n_problems);
    int64_t rows = 0;
    for (int32_t p = 0; p < n_problems; ++p) {
        const int64_t K = obs_offsets[p + 1] - obs_offsets[p];
        if (K < 1 || K > IOD_MAX_OBS)
            return bail(fail(IOD_EINVAL, "problem %d: %lld observations", p, (long long)K));
        const bool ranged = obs_ranges && sigma_range[p] != 0.0;
        int rc = make_problem(mu[p], chief_states + 6 * (size_t)p, obs_times + obs_offsets[p],
                              obs_angles + 2 * obs_offsets[p],
                              ranged ? obs_ranges + obs_offsets[p] : nullptr, (int32_t)K, sigma[p],
                              ranged ? sigma_range[p] : 0.0, opt ? opt + p : nullptr, b->probs[p]);
        if (rc != IOD_OK) {
            char msg[512];
            std::snprintf(msg, sizeof msg, "%s", g_err);
            return bail(fail(rc, "problem %d: %s", p, msg));
        }
        b->tab_off[p] = rows;
        rows += K;
    }
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) return bail(hip_fail(e, "hipGetDevice"));
    std::vector<double> tab((size_t)rows * TAB_W);
    std::vector<int32_t> ns((size_t)rows);
    for (int32_t p = 0; p < n_problems; ++p) {
        std::copy(b->probs[p].tab.begin(), b->probs[p].tab.end(), tab.begin() + b->tab_off[p] * TAB_W);
        std::copy(b->probs[p].ns.begin(), b->probs[p].ns.end(), ns.begin() + b->tab_off[p]);
    }
    if ((e = hipMalloc(&b->d_tab, tab.size() * sizeof(double))) != hipSuccess)
        return bail(hip_fail(e, "hipMalloc table"));
    if ((e = hipMalloc(&b->d_ns, ns.size() * sizeof(int32_t))) != hipSuccess)
        return bail(hip_fail(e, "hipMalloc steps"));
    if ((e = hipMemcpy(b->d_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(b->d_ns, ns.data(), ns.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(hip_fail(e, "hipMemcpy tables"));
    // chief ephemerides of all problems in one launch
    std::vector<ProbDesc> descs(n_problems);
    for (int32_t p = 0; p < n_problems; ++p) descs[p] = desc_of(b->kargs(p), b->probs[p].chief, nullptr);
    DevBuf d_desc;
    if ((e = hipMalloc(&d_desc.p, descs.size() * sizeof(ProbDesc))) != hipSuccess)
        return bail(hip_fail(e, "hipMalloc descriptors"));
    if ((e = hipMemcpy(d_desc.p, descs.data(), descs.size() * sizeof(ProbDesc), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(hip_fail(e, "hipMemcpy descriptors"));
    if ((e = launch_chief(descs[0], (const ProbDesc *)d_desc.p, n_problems, nullptr)) != hipSuccess)
        return bail(hip_fail(e, "chief launch"));
    if ((e = hipDeviceSynchronize()) != hipSuccess) return bail(hip_fail(e, "chief ephemerides"));
    *out = b;
    return IOD_OK;
}

int iod_batch_destroy(iod_batch *b)
{
    if (!b) return IOD_OK;
    int rc = IOD_OK;
    if (hipSetDevice(b->device) == hipSuccess) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) rc = hip_fail(e, "hipDeviceSynchronize");
        b->graphs.clear();
        if (b->ev0) (void)hipEventDestroy(b->ev0);
        if (b->ev1) (void)hipEventDestroy(b->ev1);
        if (b->stream) (void)hipStreamDestroy(b->stream);
        b->ev0 = b->ev1 = nullptr;
        b->stream = nullptr;
        if (b->d_tab && (e = hipFree(b->d_tab)) != hipSuccess && rc == IOD_OK) rc = hip_fail(e, "hipFree");
        if (b->d_ns && (e = hipFree(b->d_ns)) != hipSuccess && rc == IOD_OK) rc = hip_fail(e, "hipFree");
    }
    delete b;
    return rc;
}

int32_t iod_batch_size(const iod_batch *b)
{
    if (!b) return fail(IOD_EINVAL, "null batch");
    return b->P;
}

int64_t iod_batch_steps(const iod_batch *b, int32_t p)
{
    if (!b) return fail(IOD_EINVAL, "null batch");
    if (p < 0 || p >= b->P) return fail(IOD_EINVAL, "problem %d out of range", p);
    return b->probs[p].steps;
}

int iod_batch_set_config(iod_batch *b, const iod_launch_config *cfg)
{
    if (!b) return fail(IOD_EINVAL, "null batch");
    int rc = check_config(cfg);
    if (rc != IOD_OK) return rc;
    b->cfg = *cfg;
    return IOD_OK;
}

int iod_batch_get_config(const iod_batch *b, iod_launch_config *cfg)
{
    if (!b || !cfg) return fail(IOD_EINVAL, "null pointer");
    *cfg = b->cfg;
    return IOD_OK;
}

int iod_batch_set_fp32_mode(iod_batch *b, int32_t mode)
{
    if (!b) return fail(IOD_EINVAL, "null batch");
    if (mode != IOD_FP32_RELATIVE && mode != IOD_FP32_ABSOLUTE)
        return fail(IOD_EINVAL, "unknown FP32 mode %d", mode);
    b->fp32_mode = mode;
    return IOD_OK;
}

int64_t iod_batch_offsets(const iod_batch *b, const int64_t *m, int64_t *off)
{
    if (!b || !m || !off) return fail(IOD_EINVAL, "null pointer");
    int64_t o = 0;
    for (int32_t p = 0; p < b->P; ++p) {
        if (m[p] < 0 || m[p] > MAX_M) return fail(IOD_EINVAL, "problem %d: m out of range", p);
        off[p] = o;
        o += round64(m[p]);
    }
    off[b->P] = o;
    return o;
}

}  // extern "C"

namespace {

// Device-side layout of one batched launch: descriptors and work list.
struct BatchLayout {
    std::vector<ProbDesc> descs;
    std::vector<int32_t> porder;  // [P] problem order of the work list
    std::vector<int32_t> work;  // [grid][2]
    int64_t ld = 0, total_slots = 0, grid = 0;
};

int batch_layout(const iod_batch *b, const iod_pso_params *params, const int64_t *m, int bs,
                 int order, BatchLayout &L)
{
    std::vector<int64_t> off(b->P + 1);
    int64_t ld = iod_batch_offsets(b, m, off.data());
    if (ld < 0) return (int)ld;
    L.ld = ld;
    L.descs.resize(b->P);
    int64_t slots = 0;
    for (int32_t p = 0; p < b->P; ++p) {
        ProbDesc &D = L.descs[p];
        D = desc_of(b->kargs(p), b->probs[p].chief, params ? params + p : nullptr);
        set_grid(D, params ? params + p : nullptr, m[p]);
        D.m = m[p];
        D.off = off[p];
        D.slot_off = slots;
        D.nslots = ceil_div(m[p], bs);
        D.block = bs;
        slots += D.nslots;
    }
    L.total_slots = slots;
    std::vector<int32_t> pord(b->P);
    std::iota(pord.begin(), pord.end(), 0);
    if (order == IOD_ORDER_LONGEST_FIRST)
        std::stable_sort(pord.begin(), pord.end(), [&](int32_t a, int32_t c) {
            return b->probs[a].steps > b->probs[c].steps;
        });
    L.porder = pord;
    L.work.clear();
    for (int32_t p : pord)
        for (int64_t t = 0; t < L.descs[p].nslots; ++t) {
            L.work.push_back(p);
            L.work.push_back((int32_t)t);
        }
    L.grid = (int64_t)L.work.size() / 2;
    if (L.grid > 0x7fffffff) return fail(IOD_EINVAL, "batch too large for one launch");
    return IOD_OK;
}

// Allocates and runs one batched solve; optional timing of the iterations.
// top_k = 0: FP64 swarm. top_k > 0: FP32 ranking with FP64 re-evaluation of
// the top_k personal bests per problem each iteration.
// Optional last stage of a batched solve: Gauss-Newton polish of each
// problem's n_cand best personal bests.
struct PolishStage {
    int32_t n_cand, n_gn;
    double *best_states, *best_chi2, *best_costs;  // host [P][6], [P], [P]
};
int polish_stage_run(iod_batch *b, const BatchLayout &L, const SwarmArrays &B,
                     const PolishStage &S, const double *final_recs, hipStream_t st);

int batch_run(iod_batch *b, const iod_pso_params *params, const int64_t *m, int64_t n_iter,
              const iod_launch_config &cfg, double *best_states, double *best_costs,
              double *history, double *iter_ms, int32_t top_k = 0,
              const PolishStage *stage = nullptr)
{
    const int bs = block_of(cfg);
    const bool rel = top_k > 0 && b->fp32_mode == IOD_FP32_RELATIVE;
    int rc = rel ? ensure_chief_tables(b) : IOD_OK;
    if (rc != IOD_OK) return rc;
    BatchLayout L;
    rc = batch_layout(b, params, m, bs, cfg.order, L);
    if (rc != IOD_OK) return rc;
    Phase swarm_phase(top_k ? "iod_batch: mixed-precision swarm" : "iod_batch: FP64 swarm");
    const int64_t P = b->P, ld = L.ld;
    const size_t nd = (size_t)(20 * ld + 2 * L.total_slots * REC + 2 * P * REC + P * (n_iter + 1) + P);
    // stream, storage and tables are the batch's, kept for the next call
    if (!b->stream) HIP_TRY(hipStreamCreate(&b->stream));
    hipStream_t st = b->stream;
    HIP_TRY(b->swarm.ensure(nd * sizeof(double)));
    if (top_k > 0) HIP_TRY(b->cand.ensure((size_t)P * top_k * sizeof(int32_t)));
    HIP_TRY(b->porder.upload(L.porder, st));
    int32_t *cand = b->cand.as<int32_t>();
    double *base = b->swarm.as<double>();
    double *hist = base + 20 * ld + 2 * L.total_slots * REC + 2 * P * REC;
    double *stop = hist + P * (n_iter + 1);
    for (int64_t p = 0; p < P; ++p) {
        L.descs[p].hist = hist + p * (n_iter + 1);
        L.descs[p].hist_len = n_iter + 1;
    }
    HIP_TRY(b->desc.upload(L.descs, st));
    HIP_TRY(b->work.upload(L.work, st));
    SwarmArrays B;
    B.desc = b->desc.as<const ProbDesc>();
    B.work = b->work.as<const int32_t>();
    B.x = base;
    B.v = base + 6 * ld;
    B.p = base + 12 * ld;
    B.jp = base + 18 * ld;
    B.cost = base + 19 * ld;
    B.slots = base + 20 * ld;
    B.recs = B.slots + 2 * L.total_slots * REC;
    B.stop = stop;
    B.porder = b->porder.as<const int32_t>();
    B.ld = ld;
    B.total_slots = L.total_slots;
    B.nprob = P;
    const ProbDesc &d0 = L.descs[0];
    // one iteration: FP64 fused launch, or FP32 launch + top-k + FP64 re-evaluation
    auto iterate = [&](int64_t n) -> hipError_t {
        if (top_k == 0) return launch_swarm_iter(d0, B, bs, L.grid, n, st, cfg.waves);
        hipError_t e = launch_mixed_iter(d0, B, bs, L.grid, n, rel, st);
        if (e == hipSuccess) e = launch_topk(B, B.jp, top_k, cand, st);
        if (e == hipSuccess) e = launch_reeval64(B, cand, top_k, n, st);
        return e;
    };
    if (top_k == 0) {
        HIP_TRY(launch_swarm_init(d0, B, bs, L.grid, st));
    } else {
        HIP_TRY(launch_mixed_init(d0, B, bs, L.grid, rel, st));
        HIP_TRY(launch_topk(B, B.jp, top_k, cand, st));
        HIP_TRY(launch_reeval64(B, cand, top_k, 0, st));
    }
    if (iter_ms) {
        if (!b->ev0) HIP_TRY(hipEventCreate(&b->ev0));
        if (!b->ev1) HIP_TRY(hipEventCreate(&b->ev1));
        // the first iteration reuses the initial evaluation: run it untimed
        HIP_TRY(iterate(1));
        HIP_TRY(hipEventRecord(b->ev0, st));
    }
    const int64_t n0 = iter_ms ? 1 : 0;
    // the graph's launches read the descriptors, work list and problem order
    // from device tables (refreshed above when they change); the key holds
    // every launch argument
    Key key;
    key.add(d0).add(B).add(bs).add(L.grid).add(cfg.waves).add(top_k).add(cand).add(rel);
    rc = run_iterations(st, cfg.graph != 0, n0, n_iter - n0, iterate, &b->graphs, key);
    if (rc == IOD_OK && iter_ms) {
        hipError_t e = hipEventRecord(b->ev1, st);
        if (e == hipSuccess) e = hipEventSynchronize(b->ev1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, b->ev0, b->ev1);
        if (e != hipSuccess) rc = hip_fail(e, "iteration timing");
        *iter_ms = n_iter > n0 ? ms / (double)(n_iter - n0) : 0.0;
    }
    if (rc == IOD_OK && top_k == 0) {
        hipError_t e = launch_swarm_final(d0, B, n_iter, st);
        if (e != hipSuccess) rc = hip_fail(e, "final launch");
    }
    if (rc == IOD_OK && stage) {
        HIP_TRY(hipStreamSynchronize(st));
        swarm_phase.end();
        Phase refine_phase("iod_batch: refinement");
        rc = polish_stage_run(b, L, B, *stage, B.recs + (n_iter & 1) * P * REC, st);
    }
    if (rc == IOD_OK && (best_states || best_costs)) {
        std::vector<double> recs((size_t)P * REC);
        hipError_t e = hipMemcpyAsync(recs.data(), B.recs + (n_iter & 1) * P * REC, recs.size() * sizeof(double),
                                      hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "read-back");
        for (int64_t p = 0; p < P; ++p) {
            if (best_states) std::memcpy(best_states + 6 * p, &recs[p * REC + 2], 6 * sizeof(double));
            if (best_costs) best_costs[p] = recs[p * REC];
        }
    }
    if (rc == IOD_OK && history) {
        hipError_t e = hipMemcpyAsync(history, hist, (size_t)P * (n_iter + 1) * sizeof(double),
                                      hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "history read-back");
    }
    hipError_t e = hipStreamSynchronize(st);
    if (rc == IOD_OK && e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
    return rc;
}

int check_batch_swarm_args(const iod_batch *b, const iod_pso_params *params, const int64_t *m)
{
    if (!params || !m) return fail(IOD_EINVAL, "null host pointer");
    for (int32_t p = 0; p < b->P; ++p) {
        if (m[p] < 1 || m[p] > MAX_M) return fail(IOD_EINVAL, "problem %d: m out of range", p);
        int rc = check_pso(params + p);
        if (rc != IOD_OK) {
            char msg[512];
            std::snprintf(msg, sizeof msg, "%s", g_err);
            return fail(rc, "problem %d: %s", p, msg);
        }
    }
    return IOD_OK;
}

int batch_eval_impl(iod_batch *b, const double *x, int64_t ld, const int64_t *m, double *cost,
                    void *stream, bool f32);

}  // namespace

extern "C" {

int iod_batch_eval(iod_batch *b, const double *x, int64_t ld, const int64_t *m, double *cost,
                   void *stream)
{
    return batch_eval_impl(b, x, ld, m, cost, stream, false);
}

int iod_batch_eval_f32(iod_batch *b, const double *x, int64_t ld, const int64_t *m, double *cost,
                       void *stream)
{
    return batch_eval_impl(b, x, ld, m, cost, stream, true);
}

int iod_propagate_f32(iod_handle *h, const double *x, int64_t ld, int64_t m, double *states,
                      void *stream)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_swarm_view(x, ld, m, states);
    if (rc != IOD_OK || m == 0) return rc;
    const bool rel = h->fp32_mode == IOD_FP32_RELATIVE;
    if (rel) rc = ensure_chief_tables(h);
    if (rc != IOD_OK) return rc;
    HIP_TRY(launch_propagate32(h->kargs(), x, ld, m, states, rel, (hipStream_t)stream));
    return IOD_OK;
}

int iod_batch_select_topk(iod_batch *b, const double *keys, int64_t ld, const int64_t *m,
                          int32_t top_k, int32_t *out, void *stream)
{
    int rc = check_batch(b);
    if (rc != IOD_OK) return rc;
    if (!m) return fail(IOD_EINVAL, "null m");
    if (top_k < 1 || top_k > TOPK_MAX) return fail(IOD_EINVAL, "top_k must lie in [1, %d]", TOPK_MAX);
    BatchLayout L;
    rc = batch_layout(b, nullptr, m, 256, b->cfg.order, L);
    if (rc != IOD_OK) return rc;
    if (ld < L.ld) return fail(IOD_EINVAL, "ld = %lld < %lld", (long long)ld, (long long)L.ld);
    if (!keys || !out) return fail(IOD_EINVAL, "null device pointer");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(b->topk_desc.upload(L.descs, st));
    SwarmArrays B;
    std::memset(&B, 0, sizeof B);
    B.desc = b->topk_desc.as<const ProbDesc>();
    B.ld = ld;
    B.nprob = b->P;
    HIP_TRY(launch_topk(B, keys, top_k, out, st));
    return IOD_OK;
}

int iod_batch_solve_mixed(iod_batch *b, const iod_pso_params *params, const int64_t *m,
                          int64_t n_iter, int32_t top_k, double *best_states, double *best_costs,
                          double *history)
{
    int rc = check_batch(b);
    if (rc == IOD_OK) rc = check_batch_swarm_args(b, params, m);
    if (rc != IOD_OK) return rc;
    if (n_iter < 0) return fail(IOD_EINVAL, "n_iter < 0");
    if (top_k < 1 || top_k > TOPK_MAX) return fail(IOD_EINVAL, "top_k must lie in [1, %d]", TOPK_MAX);
    b->last_iter_ms = 0.0;
    return batch_run(b, params, m, n_iter, b->cfg, best_states, best_costs, history,
                     n_iter >= 2 ? &b->last_iter_ms : nullptr, top_k);
}

}  // extern "C"

namespace {

int batch_eval_impl(iod_batch *b, const double *x, int64_t ld, const int64_t *m, double *cost,
                    void *stream, bool f32)
{
    int rc = check_batch(b);
    if (rc != IOD_OK) return rc;
    if (!m) return fail(IOD_EINVAL, "null m");
    const int bs = block_of(b->cfg);
    BatchLayout L;
    rc = batch_layout(b, nullptr, m, bs, b->cfg.order, L);
    if (rc != IOD_OK) return rc;
    if (ld < L.ld) return fail(IOD_EINVAL, "ld = %lld < %lld", (long long)ld, (long long)L.ld);
    if (L.grid == 0) return IOD_OK;
    if (!x || !cost) return fail(IOD_EINVAL, "null device pointer");
    const bool rel = b->fp32_mode == IOD_FP32_RELATIVE;
    if (f32 && rel && !b->chief_built) {
        rc = ensure_chief_tables(b);
        if (rc != IOD_OK) return rc;
        rc = batch_layout(b, nullptr, m, bs, b->cfg.order, L);
        if (rc != IOD_OK) return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    // the launch tables are the batch's, copied only when they change, so the
    // call returns without waiting for the device
    HIP_TRY(b->eval_desc.upload(L.descs, st));
    HIP_TRY(b->eval_work.upload(L.work, st));
    SwarmArrays B;
    std::memset(&B, 0, sizeof B);
    B.desc = b->eval_desc.as<const ProbDesc>();
    B.work = b->eval_work.as<const int32_t>();
    B.x = const_cast<double *>(x);
    B.cost = cost;
    B.ld = ld;
    B.nprob = b->P;
    B.total_slots = L.total_slots;
    if (f32)
        HIP_TRY(launch_eval32(L.descs[0], B, bs, L.grid, rel, st));
    else
        HIP_TRY(launch_eval(L.descs[0], B, bs, L.grid, st));
    return IOD_OK;
}

}  // namespace

extern "C" {

int iod_batch_solve(iod_batch *b, const iod_pso_params *params, const int64_t *m, int64_t n_iter,
                    double *best_states, double *best_costs, double *history)
{
    int rc = check_batch(b);
    if (rc == IOD_OK) rc = check_batch_swarm_args(b, params, m);
    if (rc != IOD_OK) return rc;
    if (n_iter < 0) return fail(IOD_EINVAL, "n_iter < 0");
    b->last_iter_ms = 0.0;
    return batch_run(b, params, m, n_iter, b->cfg, best_states, best_costs, history,
                     n_iter >= 2 ? &b->last_iter_ms : nullptr);
}

double iod_batch_last_iter_ms(const iod_batch *b)
{
    if (!b) return fail(IOD_EINVAL, "null batch");
    return b->last_iter_ms;
}

int iod_batch_autotune(iod_batch *b, const iod_pso_params *params, const int64_t *m,
                       int64_t trial_iters, int32_t top_k, iod_launch_config *chosen,
                       double *ms_per_iter, int32_t *n_candidates)
{
    int rc = check_batch(b);
    if (rc == IOD_OK) rc = check_batch_swarm_args(b, params, m);
    if (rc != IOD_OK) return rc;
    if (trial_iters < 2) return fail(IOD_EINVAL, "trial_iters must be >= 2");
    if (top_k < 0 || top_k > TOPK_MAX) return fail(IOD_EINVAL, "top_k must lie in [0, %d]", TOPK_MAX);
    Phase phase("iod_batch_autotune");
    const int blocks[3] = {64, 128, 256};
    // the occupancy choice applies to the FP64 iteration kernel only
    const int n_waves = top_k == 0 ? 2 : 1;
    const int waves_of[2] = {0, 3};
    iod_launch_config best{256, IOD_ORDER_LONGEST_FIRST, 1, 0};
    double best_ms = INFINITY;
    int32_t c = 0;
    for (int wi = 0; wi < n_waves; ++wi)
        for (int bi = 0; bi < 3; ++bi)
            for (int order = 0; order < 2; ++order)
                for (int graph = 0; graph < 2; ++graph) {
                    iod_launch_config cfg{blocks[bi], order, graph, waves_of[wi]};
                    double ms = 0;
                    rc = batch_run(b, params, m, trial_iters, cfg, nullptr, nullptr, nullptr, &ms,
                                   top_k);
                    if (rc != IOD_OK) return rc;
                    if (ms_per_iter) ms_per_iter[c] = ms;
                    ++c;
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = cfg;
                    }
                }
    if (n_candidates) *n_candidates = c;
    b->cfg = best;
    if (chosen) *chosen = best;
    return IOD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Sensitivities and the Gauss-Newton polish
// ---------------------------------------------------------------------------

namespace {

// Adjoint scratch rows (of 6 doubles per column) for one problem.
int64_t adj_rows(const HostProblem &P)
{
    const int64_t S = P.ns[P.K - 1];
    return (S + ADJ_CKPT - 1) / ADJ_CKPT + ADJ_CKPT;
}

// Doubles of polish workspace per column besides the adjoint rows:
// jtj 21, jtr 6, grad 6, trial 6, chi2 at trial 1, damping 1, cost 1.
constexpr int64_t POLISH_COLS = 42;

// Damped Gauss-Newton on the columns of B.x (in place): the normal matrix
// from the forward tangent, the gradient from the discrete adjoint; d0 / the
// descriptors in B must carry the least-squares cost (mode 1).
int polish_run(const ProbDesc &d0, SwarmArrays B, int bs, int64_t grid, int32_t n_iter,
               double *chi2, double *work, int64_t ld, hipStream_t st)
{
    double *jtj = work;
    double *jtr = jtj + 21 * ld;
    double *g = jtr + 6 * ld;
    double *xt = g + 6 * ld;
    double *chi2t = xt + 6 * ld;
    double *lam = chi2t + ld;
    double *cost = lam + ld;
    double *adj = cost + ld;
    double *x = B.x;
    HIP_TRY(launch_fill_cols(d0, B, bs, grid, lam, 1e-3, st));
    for (int32_t it = 0; it < n_iter; ++it) {
        B.x = x;
        HIP_TRY(launch_normal(d0, B, bs, grid, chi2, jtj, jtr, st));
        B.cost = cost;
        HIP_TRY(launch_grad(d0, B, bs, grid, g, adj, ld, 1, st));
        HIP_TRY(launch_gn_solve(d0, B, bs, grid, jtj, g, 0.5, lam, xt, st));
        B.x = xt;
        B.cost = chi2t;
        HIP_TRY(launch_eval(d0, B, bs, grid, st));
        B.x = x;
        HIP_TRY(launch_gn_accept(d0, B, bs, grid, xt, chi2, chi2t, lam, st));
    }
    if (n_iter == 0) {
        B.x = x;
        HIP_TRY(launch_normal(d0, B, bs, grid, chi2, jtj, jtr, st));
    }
    return IOD_OK;
}

// The batched refinement loop: each iteration forms the normal equations and
// the adjoint gradient of every live candidate (packed: lanes lists the
// (problem, candidate) pairs, several problems to a wave), tries T dampings
// per candidate side by side (one wave per problem, in the lanes that the
// candidates leave free), adds the geodesic correction, keeps the best
// trial, and retires problems whose candidates have all stopped moving. PB
// holds the candidate columns (p * 64 + j, j < n[p]); tdesc the trial
// descriptors (n[p] * T columns); jrows the candidates' rows of J.
constexpr double POLISH_STEP_TOL = 1e-12;

constexpr double GN_FINAL_MAX_STEP = 1e-6;  // largest component of a final undamped step
constexpr double GEO_HD = 0.1;      // finite-difference step along v, as a fraction of v
constexpr double GEO_ALPHA = 0.75;  // accept the correction a if 2 |a| <= alpha |v|

int polish_trials_run(const ProbDesc &d0, SwarmArrays PB, const ProbDesc *tdesc,
                      const int32_t *n, int64_t P, int32_t T, int32_t n_iter, double *chi2,
                      double *work, double *vt, double *jrows, int32_t n_cand, int32_t *active,
                      int32_t *done, const int32_t *lanes, int64_t nlanes, int32_t *live,
                      int64_t *live_count, int64_t ld, hipStream_t st)
{
    const int64_t jld = P * n_cand;
    double *jtj = work;
    double *jtr = jtj + 21 * ld;
    double *g = jtr + 6 * ld;
    double *xt = g + 6 * ld;
    double *chi2t = xt + 6 * ld;
    double *lam = chi2t + ld;
    double *cost = lam + ld;
    double *adj = cost + ld;
    double *x = PB.x;
    PB.active = active;
    HIP_TRY(launch_fill_cols(d0, PB, 64, P, lam, 1e-3, st));
    SwarmArrays TB = PB;
    TB.desc = tdesc;
    TB.x = xt;
    TB.cost = chi2t;
    // the normal equations and the gradient see only the candidates: packed,
    // several problems' candidates to a wave, problems with the most RK4
    // steps first. Each iteration they take only the live pairs (problem
    // active, candidate not done), compacted in that order after the select
    // step, so retired pairs leave the waves; the grid stays that of all
    // pairs and the waves past the live count exit at once. Both sweeps go
    // in one launch, so that the tangent and the adjoint sweep of the last
    // live pairs run at the same time.
    Lanes KL;
    KL.pairs = lanes;
    KL.n = nlanes;
    Lanes LL;
    LL.pairs = live;
    LL.n = nlanes;
    LL.count = live_count;
    const int64_t kgrid = (nlanes + 63) / 64;
    HIP_TRY(launch_live_lanes(lanes, nlanes, active, done, live, live_count, st));
    for (int32_t it = 0; it < n_iter; ++it) {
        SwarmArrays GB = PB;
        GB.cost = cost;
        HIP_TRY(launch_normal_grad(d0, PB, GB, kgrid, chi2, jtj, jtr, jrows, n_cand, jld, g, adj,
                                   ld, 1, st, LL));
        HIP_TRY(launch_gn_trials(x, jtj, g, lam, n, active, done, T, P, ld, xt, vt, st));
        HIP_TRY(launch_geo(PB.desc, x, jtj, jtr, jrows, n_cand, jld, lam, n, active, done, T, P,
                           ld, GEO_HD, GEO_ALPHA, vt, xt, st));
        HIP_TRY(launch_eval(d0, TB, 64, P, st));
        HIP_TRY(launch_gn_select(x, chi2, lam, done, active, xt, chi2t, n, T, P, ld,
                                 POLISH_STEP_TOL, st));
        if (it + 1 < n_iter)
            HIP_TRY(launch_live_lanes(lanes, nlanes, active, done, live, live_count, st));
    }
    if (n_iter == 0) {
        HIP_TRY(launch_normal(d0, PB, 64, P, chi2, jtj, jtr, st));
        return IOD_OK;
    }
    // Every candidate, retired or not, then takes up to two undamped
    // Gauss-Newton steps where they are small (the second removes what the
    // first leaves of the residuals' curvature): near the minimum the damped
    // iterations stop where binary64 chi2 noise hides the remaining decrease
    // along weakly observed directions, while the step itself, from the
    // normal equations, still resolves the minimiser. chi2 is then evaluated
    // at the final states.
    SwarmArrays AB = PB;
    AB.active = nullptr;
    for (int f = 0; f < 2; ++f) {
        HIP_TRY(launch_normal(d0, AB, 64, kgrid, chi2, jtj, jtr, st, nullptr, 0, 0, KL));
        HIP_TRY(launch_gn_final(x, jtj, jtr, n, P, ld, GN_FINAL_MAX_STEP, st));
    }
    AB.cost = chi2;
    HIP_TRY(launch_eval(d0, AB, 64, P, st));
    return IOD_OK;
}

int polish_stage_run(iod_batch *b, const BatchLayout &L, const SwarmArrays &B,
                     const PolishStage &S, const double *final_recs, hipStream_t st)
{
    const int64_t P = b->P, stride = 64, ldp = P * stride;
    int64_t rows = 0;
    for (const HostProblem &Pb : b->probs) rows = std::max(rows, adj_rows(Pb));
    // trials per candidate: the free lanes of the problem's 64-lane wave, at most 8
    const int32_t T = std::max(1, std::min(8, 64 / S.n_cand));
    // rows of J of every candidate: max over problems of K R (R = 3 with ranges, else 2)
    int64_t jrow_max = 0;
    for (const HostProblem &Pb : b->probs)
        jrow_max = std::max<int64_t>(jrow_max, (int64_t)Pb.K * (Pb.sigma_range > 0 ? 3 : 2));
    // the stage's buffers are the batch's, grown when needed and kept
    PolishBuffers &Q = b->pol;
    HIP_TRY(Q.cand.ensure((size_t)P * S.n_cand * sizeof(int32_t)));
    HIP_TRY(Q.x.ensure((size_t)6 * ldp * sizeof(double)));
    HIP_TRY(Q.chi.ensure((size_t)ldp * sizeof(double)));
    HIP_TRY(Q.work.ensure((size_t)(POLISH_COLS + rows * 6) * ldp * sizeof(double)));
    HIP_TRY(Q.best.ensure((size_t)6 * P * sizeof(double)));
    HIP_TRY(Q.bchi.ensure((size_t)P * sizeof(double)));
    HIP_TRY(Q.cost.ensure((size_t)P * sizeof(double)));
    HIP_TRY(Q.act.ensure((size_t)P * sizeof(int32_t)));
    HIP_TRY(Q.done.ensure((size_t)ldp * sizeof(int32_t)));
    HIP_TRY(Q.vt.ensure((size_t)6 * ldp * sizeof(double)));
    HIP_TRY(Q.jrows.ensure((size_t)jrow_max * 6 * P * S.n_cand * sizeof(double)));
    // candidates: each problem's global best, then its best personal bests
    // (in the mixed-precision swarm the first is decided by FP64 costs, the
    // ranking of the others by FP32 costs)
    HIP_TRY(launch_topk(B, B.jp, S.n_cand, Q.cand.as<int32_t>(), st));
    HIP_TRY(launch_gather(B, Q.cand.as<const int32_t>(), S.n_cand, final_recs, Q.x.as<double>(),
                          ldp, stride, st));
    std::vector<ProbDesc> pd(L.descs), ed(L.descs), td(L.descs);
    std::vector<int32_t> list(2 * P), n(P);
    for (int64_t p = 0; p < P; ++p) {
        ProbDesc &D = pd[p];
        D.m = std::min<int64_t>(S.n_cand, L.descs[p].m);
        D.off = p * stride;
        D.slot_off = 0;
        D.nslots = 1;
        D.block = 64;
        D.hist = nullptr;
        D.hist_len = 0;
        D.k.mode = IOD_COST_CHI2;
        td[p] = D;
        td[p].m = D.m * T;
        if (td[p].m > stride) return fail(IOD_EINVAL, "trial columns exceed the stride");
        ed[p] = D;
        ed[p].k.mode = L.descs[p].k.mode;
        ed[p].m = 1;
        ed[p].off = p;
        list[2 * p] = (int32_t)p;
        list[2 * p + 1] = 0;
        n[p] = (int32_t)D.m;
    }
    HIP_TRY(Q.desc.upload(pd, st));
    HIP_TRY(Q.edesc.upload(ed, st));
    HIP_TRY(Q.list.upload(list, st));
    HIP_TRY(Q.nn.upload(n, st));
    HIP_TRY(Q.tdesc.upload(td, st));
    // packed lanes: (problem, candidate), problems with the most RK4 steps first
    std::vector<int32_t> by_steps(P);
    std::iota(by_steps.begin(), by_steps.end(), 0);
    std::stable_sort(by_steps.begin(), by_steps.end(), [&](int32_t a, int32_t c) {
        return b->probs[a].steps > b->probs[c].steps;
    });
    std::vector<int32_t> lanes;
    lanes.reserve((size_t)2 * P * S.n_cand);
    for (int32_t p : by_steps)
        for (int32_t j = 0; j < n[p]; ++j) {
            lanes.push_back(p);
            lanes.push_back(j);
        }
    const int64_t nlanes = (int64_t)lanes.size() / 2;
    HIP_TRY(Q.lanes.upload(lanes, st));
    HIP_TRY(Q.live.ensure(std::max<size_t>(lanes.size(), 2) * sizeof(int32_t)));
    HIP_TRY(Q.live_count.ensure(sizeof(int64_t)));
    // the retirement flags start cleared on every call (the kernels change them)
    HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)Q.act.p, 1, (size_t)P, st));
    HIP_TRY(hipMemsetAsync(Q.done.p, 0, (size_t)ldp * sizeof(int32_t), st));
    SwarmArrays PB;
    std::memset(&PB, 0, sizeof PB);
    PB.desc = Q.desc.as<const ProbDesc>();
    PB.work = Q.list.as<const int32_t>();
    PB.x = Q.x.as<double>();
    PB.ld = ldp;
    PB.nprob = P;
    int rc = polish_trials_run(pd[0], PB, Q.tdesc.as<const ProbDesc>(), Q.nn.as<const int32_t>(), P,
                               T, S.n_gn, Q.chi.as<double>(), Q.work.as<double>(),
                               Q.vt.as<double>(), Q.jrows.as<double>(), S.n_cand,
                               Q.act.as<int32_t>(), Q.done.as<int32_t>(),
                               Q.lanes.as<const int32_t>(), nlanes, Q.live.as<int32_t>(),
                               Q.live_count.as<int64_t>(), ldp, st);
    if (rc != IOD_OK) return rc;
    HIP_TRY(launch_pick_best(Q.x.as<const double>(), Q.chi.as<const double>(),
                             Q.nn.as<const int32_t>(), P, ldp, stride, Q.best.as<double>(),
                             Q.bchi.as<double>(), st));
    // the problem's own cost of each polished best
    SwarmArrays EB;
    std::memset(&EB, 0, sizeof EB);
    EB.desc = Q.edesc.as<const ProbDesc>();
    EB.work = Q.list.as<const int32_t>();
    EB.x = Q.best.as<double>();
    EB.cost = Q.cost.as<double>();
    EB.ld = P;
    EB.nprob = P;
    HIP_TRY(launch_eval(ed[0], EB, 64, P, st));
    std::vector<double> best(6 * P), bchi(P), bcost(P);
    HIP_TRY(hipMemcpyAsync(best.data(), Q.best.p, best.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(bchi.data(), Q.bchi.p, bchi.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(bcost.data(), Q.cost.p, bcost.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int64_t p = 0; p < P; ++p) {
        for (int d = 0; d < 6; ++d) S.best_states[6 * p + d] = best[d * P + p];
        if (S.best_chi2) S.best_chi2[p] = bchi[p];
        if (S.best_costs) S.best_costs[p] = bcost[p];
    }
    return IOD_OK;
}

// Single-problem view of m columns of x.
void single_cols(const iod_handle *h, const double *x, int64_t ld, int64_t m, int bs,
                 ProbDesc &D, SwarmArrays &B)
{
    D = desc_of(h->kargs(), h->P.chief, nullptr);
    D.m = m;
    D.nslots = ceil_div(m, bs);
    D.block = bs;
    std::memset(&B, 0, sizeof B);
    B.x = const_cast<double *>(x);
    B.ld = ld;
    B.nprob = 1;
}

// Static device scratch of iod_grad_noalloc (adjoint checkpoints and segment
// states), for callers that cannot allocate. Each device holds its own copy
// from module load until the process ends. In host code `scratch` names only
// a host-side stand-in: its device address comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address is
// ever handed to a kernel.
static __device__ __align__(256) double scratch[IOD_NOALLOC_SCRATCH_DOUBLES];

constexpr int NOALLOC_MAX_DEVICES = 64;

int noalloc_scratch(int device, double **out)
{
    static std::mutex mu;
    static double *addr[NOALLOC_MAX_DEVICES] = {};
    if (device < 0 || device >= NOALLOC_MAX_DEVICES)
        return fail(IOD_EDEVICE, "device %d beyond the %d the static scratch tracks", device,
                    NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(IOD_EDEVICE, "hipGetSymbolAddress(scratch) gave a null address");
        addr[device] = (double *)p;
    }
    *out = addr[device];
    return IOD_OK;
}

int batch_predict_impl(iod_batch *b, const double *x, double *out, bool ranges)
{
    int rc = check_batch(b);
    if (rc != IOD_OK) return rc;
    if (!x || !out) return fail(IOD_EINVAL, "null host pointer");
    const int64_t P = b->P;
    for (int64_t p = 0; p < P; ++p)
        if (!finite6(x + 6 * p)) return fail(IOD_EINVAL, "problem %lld: non-finite state", (long long)p);
    const int64_t rows = b->tab_off[P - 1] + b->probs[P - 1].K;
    const int64_t per_row = ranges ? 1 : 2;
    std::vector<ProbDesc> descs(P);
    for (int64_t p = 0; p < P; ++p) descs[p] = desc_of(b->kargs((int32_t)p), b->probs[p].chief, nullptr);
    DevBuf dd, dx, doff, dout;
    HIP_TRY(hipMalloc(&dd.p, P * sizeof(ProbDesc)));
    HIP_TRY(hipMalloc(&dx.p, 6 * P * sizeof(double)));
    HIP_TRY(hipMalloc(&doff.p, P * sizeof(int64_t)));
    HIP_TRY(hipMalloc(&dout.p, per_row * rows * sizeof(double)));
    HIP_TRY(hipMemcpy(dd.p, descs.data(), P * sizeof(ProbDesc), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dx.p, x, 6 * P * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(doff.p, b->tab_off.data(), P * sizeof(int64_t), hipMemcpyHostToDevice));
    if (ranges)
        HIP_TRY(launch_predict_ranges_batch((const ProbDesc *)dd.p, P, (const double *)dx.p,
                                            (const int64_t *)doff.p, (double *)dout.p, nullptr));
    else
        HIP_TRY(launch_predict_batch((const ProbDesc *)dd.p, P, (const double *)dx.p,
                                     (const int64_t *)doff.p, (double *)dout.p, nullptr));
    HIP_TRY(hipMemcpy(out, dout.p, per_row * rows * sizeof(double), hipMemcpyDeviceToHost));
    return IOD_OK;
}

}  // namespace

extern "C" {

int iod_batch_predict(iod_batch *b, const double *x, double *angles)
{
    return batch_predict_impl(b, x, angles, false);
}

int iod_batch_predict_ranges(iod_batch *b, const double *x, double *ranges)
{
    return batch_predict_impl(b, x, ranges, true);
}

int64_t iod_grad_work_len(const iod_handle *h, int64_t ld)
{
    if (!h) return fail(IOD_EINVAL, "null handle");
    if (ld < 1 || ld > MAX_M) return fail(IOD_EINVAL, "ld out of range");
    const int64_t per_col = adj_rows(h->P) * 6;
    if (ld > INT64_MAX / per_col) return fail(IOD_EINVAL, "workspace size overflows");
    return per_col * ld;
}

int iod_grad(iod_handle *h, const double *x, int64_t ld, int64_t m, double *cost, double *grad,
             double *work, void *stream)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_swarm_view(x, ld, m, cost);
    if (rc != IOD_OK || m == 0) return rc;
    if (!grad || !work) return fail(IOD_EINVAL, "null device pointer");
    const int bs = block_of(h->cfg);
    ProbDesc D;
    SwarmArrays B;
    single_cols(h, x, ld, m, bs, D, B);
    B.cost = cost;
    HIP_TRY(launch_grad(D, B, bs, D.nslots, grad, work, ld, -1, (hipStream_t)stream));
    return IOD_OK;
}

int iod_grad_noalloc(iod_handle *h, const double *x, int64_t ld, int64_t m, double *cost,
                     double *grad, void *stream)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_swarm_view(x, ld, m, cost);
    if (rc != IOD_OK || m == 0) return rc;
    if (!grad) return fail(IOD_EINVAL, "null device pointer");
    const int64_t per_col = adj_rows(h->P) * 6;
    if (ld > IOD_NOALLOC_SCRATCH_DOUBLES / per_col)
        return fail(IOD_EINVAL,
                    "iod_grad_noalloc: %lld doubles of adjoint scratch (ld = %lld) exceed the "
                    "static scratch of %lld doubles; use iod_grad with a workspace",
                    (long long)per_col * (long long)ld, (long long)ld,
                    (long long)IOD_NOALLOC_SCRATCH_DOUBLES);
    double *work = nullptr;
    rc = noalloc_scratch(h->device, &work);
    if (rc != IOD_OK) return rc;
    const int bs = block_of(h->cfg);
    ProbDesc D;
    SwarmArrays B;
    single_cols(h, x, ld, m, bs, D, B);
    B.cost = cost;
    HIP_TRY(launch_grad(D, B, bs, D.nslots, grad, work, ld, -1, (hipStream_t)stream));
    return IOD_OK;
}

int iod_normal_eq(iod_handle *h, const double *x, int64_t ld, int64_t m, double *chi2,
                  double *jtj, double *jtr, void *stream)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_swarm_view(x, ld, m, chi2);
    if (rc != IOD_OK || m == 0) return rc;
    if (!jtj || !jtr) return fail(IOD_EINVAL, "null device pointer");
    const int bs = block_of(h->cfg);
    ProbDesc D;
    SwarmArrays B;
    single_cols(h, x, ld, m, bs, D, B);
    HIP_TRY(launch_normal(D, B, bs, D.nslots, chi2, jtj, jtr, (hipStream_t)stream));
    return IOD_OK;
}

int64_t iod_polish_work_len(const iod_handle *h, int64_t ld)
{
    if (!h) return fail(IOD_EINVAL, "null handle");
    if (ld < 1 || ld > MAX_M) return fail(IOD_EINVAL, "ld out of range");
    return (POLISH_COLS + adj_rows(h->P) * 6) * ld;
}

int iod_polish(iod_handle *h, double *x, int64_t ld, int64_t m, int32_t n_iter, double *chi2,
               double *work, void *stream)
{
    int rc = check_handle(h);
    if (rc == IOD_OK) rc = check_swarm_view(x, ld, m, chi2);
    if (rc != IOD_OK || m == 0) return rc;
    if (!work) return fail(IOD_EINVAL, "null workspace");
    if (n_iter < 0) return fail(IOD_EINVAL, "n_iter < 0");
    const int bs = block_of(h->cfg);
    ProbDesc D;
    SwarmArrays B;
    single_cols(h, x, ld, m, bs, D, B);
    D.k.mode = IOD_COST_CHI2;
    return polish_run(D, B, bs, D.nslots, n_iter, chi2, work, ld, (hipStream_t)stream);
}

int64_t iod_batch_polish_work_len(const iod_batch *b, int64_t ld)
{
    if (!b) return fail(IOD_EINVAL, "null batch");
    if (ld < 1 || ld > MAX_M) return fail(IOD_EINVAL, "ld out of range");
    int64_t rows = 0;
    for (const HostProblem &P : b->probs) rows = std::max(rows, adj_rows(P));
    return (POLISH_COLS + rows * 6) * ld;
}

int iod_batch_polish(iod_batch *b, double *x, int64_t ld, const int64_t *m, int32_t n_iter,
                     double *chi2, double *work, void *stream)
{
    int rc = check_batch(b);
    if (rc != IOD_OK) return rc;
    if (!m) return fail(IOD_EINVAL, "null m");
    if (n_iter < 0) return fail(IOD_EINVAL, "n_iter < 0");
    const int bs = block_of(b->cfg);
    BatchLayout L;
    rc = batch_layout(b, nullptr, m, bs, b->cfg.order, L);
    if (rc != IOD_OK) return rc;
    if (ld < L.ld) return fail(IOD_EINVAL, "ld = %lld < %lld", (long long)ld, (long long)L.ld);
    if (L.grid == 0) return IOD_OK;
    if (!x || !chi2 || !work) return fail(IOD_EINVAL, "null device pointer");
    for (ProbDesc &D : L.descs) D.k.mode = IOD_COST_CHI2;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(b->bpol_desc.upload(L.descs, st));
    HIP_TRY(b->bpol_work.upload(L.work, st));
    SwarmArrays B;
    std::memset(&B, 0, sizeof B);
    B.desc = b->bpol_desc.as<const ProbDesc>();
    B.work = b->bpol_work.as<const int32_t>();
    B.x = x;
    B.ld = ld;
    B.nprob = b->P;
    return polish_run(L.descs[0], B, bs, L.grid, n_iter, chi2, work, ld, st);
}

// PSO (FP64 or mixed precision), then the Gauss-Newton polish of n_cand
// candidates per problem (its global best and its best other personal
// bests), keeping the best polished candidate.
int iod_batch_solve_polished(iod_batch *b, const iod_pso_params *params, const int64_t *m,
                             int64_t n_iter, int32_t top_k, int32_t n_cand, int32_t n_gn,
                             double *best_states, double *best_chi2, double *best_costs)
{
    int rc = check_batch(b);
    if (rc == IOD_OK) rc = check_batch_swarm_args(b, params, m);
    if (rc != IOD_OK) return rc;
    if (n_iter < 0 || n_gn < 0) return fail(IOD_EINVAL, "negative iteration count");
    if (top_k < 0 || top_k > TOPK_MAX) return fail(IOD_EINVAL, "top_k must lie in [0, %d]", TOPK_MAX);
    if (n_cand < 1 || n_cand > 64) return fail(IOD_EINVAL, "n_cand must lie in [1, 64]");
    if (!best_states) return fail(IOD_EINVAL, "null best_states");
    b->last_iter_ms = 0.0;
    PolishStage stage{n_cand, n_gn, best_states, best_chi2, best_costs};
    return batch_run(b, params, m, n_iter, b->cfg, nullptr, nullptr, nullptr,
                     n_iter >= 2 ? &b->last_iter_ms : nullptr, top_k, &stage);
}

}  // extern "C"
