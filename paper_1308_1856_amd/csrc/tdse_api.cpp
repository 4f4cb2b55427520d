// C ABI of the TDSE library: context, tables, workspace layout, launches.
// The declarations and their documentation are in include/tdse.h.
#include "tdse.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "host_eigen.hpp"
#include "tdse_internal.hpp"

using namespace tdse;

namespace {

constexpr int kEtabSteps = 256;          // steps per uploaded chunk of per-step scalars
constexpr size_t kAlign = 256;
constexpr int kTileRows = 32;            // largest number of rows per tile
constexpr int kTargetTiles = 2048;       // aim for >= 8 workgroups per CU on 256 CUs

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

const char* kTimedNames[] = {"taylor_term", "rk4_stage", "observables", "lanczos_sweep_a", "apply_h",
                             "taylor_fused", "rk4_fused"};
constexpr int kNumTimed = 7;

}  // namespace

namespace {

// Butcher tableaux of the explicit Runge-Kutta methods of the appendix
// "Runge-Kutta" (the published ones): b are the weights of the solution
// carried forward (the higher order of a pair), bhat those of the embedded
// solution (all zero without one).
struct RkTableau {
    int stages;
    double c[kRkMax];
    double a[kRkMax][kRkMax];
    double b[kRkMax];
    double bhat[kRkMax];
};
const RkTableau* rk_tableau(int method)
{
    static const RkTableau tabs[] = {
        // Euler
        {1, {0}, {{0}}, {1.0}, {0}},
        // classic fourth order
        {4, {0, 0.5, 0.5, 1.0},
         {{0}, {0.5}, {0, 0.5}, {0, 0, 1.0}},
         {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6}, {0}},
        // Fehlberg 4(5): b of order 5, bhat of order 4
        {6, {0, 1.0 / 4, 3.0 / 8, 12.0 / 13, 1.0, 1.0 / 2},
         {{0}, {1.0 / 4}, {3.0 / 32, 9.0 / 32}, {1932.0 / 2197, -7200.0 / 2197, 7296.0 / 2197},
          {439.0 / 216, -8.0, 3680.0 / 513, -845.0 / 4104},
          {-8.0 / 27, 2.0, -3544.0 / 2565, 1859.0 / 4104, -11.0 / 40}},
         {16.0 / 135, 0, 6656.0 / 12825, 28561.0 / 56430, -9.0 / 50, 2.0 / 55},
         {25.0 / 216, 0, 1408.0 / 2565, 2197.0 / 4104, -1.0 / 5, 0}},
        // Cash-Karp 5(4)
        {6, {0, 1.0 / 5, 3.0 / 10, 3.0 / 5, 1.0, 7.0 / 8},
         {{0}, {1.0 / 5}, {3.0 / 40, 9.0 / 40}, {3.0 / 10, -9.0 / 10, 6.0 / 5},
          {-11.0 / 54, 5.0 / 2, -70.0 / 27, 35.0 / 27},
          {1631.0 / 55296, 175.0 / 512, 575.0 / 13824, 44275.0 / 110592, 253.0 / 4096}},
         {37.0 / 378, 0, 250.0 / 621, 125.0 / 594, 0, 512.0 / 1771},
         {2825.0 / 27648, 0, 18575.0 / 48384, 13525.0 / 55296, 277.0 / 14336, 1.0 / 4}},
        // Dormand-Prince 5(4)
        {7, {0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0},
         {{0}, {1.0 / 5}, {3.0 / 40, 9.0 / 40}, {44.0 / 45, -56.0 / 15, 32.0 / 9},
          {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729},
          {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656},
          {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}},
         {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0},
         {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200, 187.0 / 2100, 1.0 / 40}},
        // Merson 4(3)
        {5, {0, 1.0 / 3, 1.0 / 3, 1.0 / 2, 1.0},
         {{0}, {1.0 / 3}, {1.0 / 6, 1.0 / 6}, {1.0 / 8, 0, 3.0 / 8}, {1.0 / 2, 0, -3.0 / 2, 2.0}},
         {1.0 / 6, 0, 0, 2.0 / 3, 1.0 / 6},
         {1.0 / 10, 0, 3.0 / 10, 2.0 / 5, 1.0 / 5}},
    };
    if (method < 0 || method >= (int)(sizeof tabs / sizeof tabs[0])) return nullptr;
    return &tabs[method];
}
// state-shaped work vectors of a tableau step: k_0..k_{S-2} and two g buffers
int rk_vecs(int method)
{
    const RkTableau* T = rk_tableau(method);
    return T ? T->stages + 1 : 0;
}

}  // namespace

struct tdse_ctx {
    std::string err;
    int n_inst = 0, stencil = 3, prec = 0;
    size_t elem = 16;
    std::vector<tdse_grid_desc> grids;
    std::vector<Inst> inst;
    std::vector<Tile> tiles[kNumTileSets];
    int rows_sweep = 1, rows_reduce = 1, rows_obs = 1;
    int sweep_variant = 0;              // bit 0: two radii per thread, bit 1: XCD-contiguous order,
                                        // bit 2: wave strips of one level (autotuned)
    int fuse_k = 0;                     // Horner terms per fused launch (0: one launch per term)
    int fuse_kind = 0;                  // fused kernel: 0 LDS rings, 1 wave strips, 2 pair strips,
                                        // 3 pair strips in a persistent launch over a work queue
    bool rk4_fused = true;              // RK4: one strip launch per step (else four stage launches)
    int rows_rk4 = 16;
    int rows_fused = 16;
    int64_t total_cols = 0;             // sum over instances of ceil(N/256) * (lmax+1)
    std::vector<double> kappa;
    std::vector<double> radial;            // per instance: u0 row then n_states phi rows
    std::vector<int> lmax_max;
    int64_t state_elems = 0;
    // device binding
    bool bound = false;
    char* d_state = nullptr;
    char* d_work = nullptr;
    size_t work_bytes = 0;
    hipStream_t stream = nullptr;
    // workspace layout (bytes from d_work)
    size_t off_inst = 0, off_tiles[kNumTileSets] = {0, 0, 0, 0, 0, 0, 0}, off_kappa = 0, off_radial = 0,
           off_step = 0, off_obs_tmp = 0, off_lz = 0, off_partial = 0, off_vecs = 0, fixed_bytes = 0,
           off_zero = 0, zero_bytes = 0, off_queue = 0, off_perm = 0;
    size_t partial_doubles = 0;
    std::vector<int32_t> strip_perm;    // strip tiles, longest first (the persistent launch's order)
    size_t tile_cap[kNumTileSets] = {};  // tiles each set's workspace region holds
    size_t strip_units_cap = 0;         // most strips any wave-strip tile set can hold
    // pinned staging for the per-step scalars (double buffered)
    double* h_step[2] = {nullptr, nullptr};
    hipEvent_t step_ev[2] = {nullptr, nullptr};
    bool step_ev_used[2] = {false, false};
    int step_buf = 0;
    // the observables of the Taylor path run on a second stream (default
    // priority), overlapping the next step; created on first use
    bool obs_overlap = true;
    // the Taylor path on wave strips sums the main observables in the step's
    // last launch (obs_req: where, set per step by the step loop;
    // obs_main_done: the step function did it)
    bool obs_fusion = true;
    double* obs_req = nullptr;
    bool obs_main_done = false;
    hipStream_t obs_stream = nullptr;
    hipEvent_t obs_fork = nullptr, obs_join = nullptr, obs_done[2] = {nullptr, nullptr};
    // Krylov dimension requested by the last tdse_step_lanczos call (0: none)
    int lz_m = 0;
    // the Runge-Kutta tableau whose stage times upload_steps fills in
    // (kEStage0 + i: E(t_n + c_i dt)); 0 stages for the other methods
    int rk_stages = 0;
    double rk_c[kRkMax] = {};
    // the absorbing mask (Sec. 2.1) and the flux yield (Sec. 4) after every
    // real-time step, once set for some instance (tdse_set_absorber,
    // tdse_set_flux); off_flux: the current at the last step, then the
    // accumulated yield, n_inst doubles each
    bool absorber_on = false, flux_on = false;
    size_t off_flux = 0;
    // Sec. 2 gauge of the coupling (0 length, 1 velocity: the step tables
    // carry A/c, the steps run the workgroup sweeps); a_run: A/c of each
    // instance at the start of the next step of the running call
    int gauge = 0;
    std::vector<double> a_run;
    // captured step graphs, keyed by the launch pattern of a chunk
    bool use_graphs = false;
    std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
    std::map<std::vector<int64_t>, void*> graph_end_psi;   // psi buffer after a graph's chunk
    void drop_graphs()
    {
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
        graphs.clear();
        graph_end_psi.clear();
    }
    // Gershgorin bounds already computed, keyed by (instance, |E|): the bound
    // costs one pass over the grid, too much to repeat on every step call
    mutable std::map<std::tuple<int, int, double>, double> bound_cache;
    // timing
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
    size_t ev_used = 0;
    std::vector<int> ev_kind;

    tdse_status fail(tdse_status code, const std::string& msg)
    {
        err = msg;
        return code;
    }
    tdse_status hip_fail(hipError_t e, const char* what)
    {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return TDSE_E_HIP;
    }
    SweepGeom geom(int set = kSweepTiles) const
    {
        SweepGeom g;
        g.zero_row = d_work + off_zero;
        g.inst = reinterpret_cast<const Inst*>(d_work + off_inst);
        g.tiles = reinterpret_cast<const Tile*>(d_work + off_tiles[set]);
        g.kappa = reinterpret_cast<const double*>(d_work + off_kappa);
        g.n_tiles = (int32_t)tiles[set].size();
        g.n_inst = n_inst;
        g.set = set;
        g.variant = 0;
        g.order = 0;
        g.plane = plane();
        g.gauge = gauge;
        g.pad_ = 0;
        return g;
    }
    // geometry of the H sweeps (apply_H, Taylor terms) in the tuned shape
    SweepGeom hgeom() const
    {
        if (gauge != 0) return geom(kSweepTiles);   // the velocity gauge: one radius per thread
        const bool strip = (sweep_variant & 4) != 0;
        SweepGeom g = geom(strip ? kApplyTiles : (sweep_variant & 1) ? kPairTiles : kSweepTiles);
        g.variant = strip ? 1 : (sweep_variant & 1);
        // bit 1: XCD-contiguous runs (workgroup sweeps), runs of kXcdGroup
        // tiles per XCD (strips)
        g.order = (sweep_variant & 2) ? (strip ? 2 : 1) : 0;
        return g;
    }
    double* d_step() const { return reinterpret_cast<double*>(d_work + off_step); }
    double* d_partial() const { return reinterpret_cast<double*>(d_work + off_partial); }
    double* d_radial() const { return reinterpret_cast<double*>(d_work + off_radial); }
    LanczosScalars* d_lz() const { return reinterpret_cast<LanczosScalars*>(d_work + off_lz); }
    double* d_jprev() const { return reinterpret_cast<double*>(d_work + off_flux); }
    unsigned* d_queue() const { return reinterpret_cast<unsigned*>(d_work + off_queue); }
    int32_t* d_perm() const { return reinterpret_cast<int32_t*>(d_work + off_perm); }
    double* d_yield() const { return d_jprev() + n_inst; }
    char* d_vec(int k) const { return d_work + off_vecs + (size_t)k * state_bytes(); }
    // elements per plane of a state-shaped vector with 48-bit storage (its
    // plane h then takes 8 * plane bytes, a multiple of 256, plane l 4 * plane)
    int64_t plane() const { return (int64_t)align_up((size_t)state_elems, 64); }
    size_t state_bytes() const
    {
        if (prec == TDSE_FP48) return 12 * (size_t)plane();
        return align_up((size_t)state_elems * elem, kAlign);
    }
    size_t vecs_needed(int method, int order_or_m) const
    {
        if (method == TDSE_METHOD_TAYLOR) return 2;
        if (method == TDSE_METHOD_RK4) return 3;
        if (method == TDSE_METHOD_LANCZOS) return (size_t)std::max(1, order_or_m);
        if (method == TDSE_METHOD_TUNE) return 4;
        if (method == TDSE_METHOD_RK_TABLEAU) return (size_t)rk_vecs(order_or_m);
        return 0;
    }
};

// ---------------------------------------------------------------------------
// timing helpers
// ---------------------------------------------------------------------------
namespace {

int timed_kind(const char* name)
{
    for (int k = 0; k < kNumTimed; ++k)
        if (std::strcmp(name, kTimedNames[k]) == 0) return k;
    return -1;
}

// HIP events around one launch, on the stream the launch goes to.
struct TimedLaunch {
    tdse_ctx* c;
    int kind;
    hipStream_t st;
    size_t slot = (size_t)-1;
    TimedLaunch(tdse_ctx* ctx, int k) : TimedLaunch(ctx, k, ctx->stream) {}
    TimedLaunch(tdse_ctx* ctx, int k, hipStream_t stream) : c(ctx), kind(k), st(stream)
    {
        if (!c->timing) return;
        if (c->ev_used == c->ev_pool.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
            c->ev_pool.emplace_back(a, b);
            c->ev_kind.push_back(-1);
        }
        slot = c->ev_used++;
        c->ev_kind[slot] = kind;
        (void)hipEventRecord(c->ev_pool[slot].first, st);
    }
    ~TimedLaunch()
    {
        if (slot != (size_t)-1) (void)hipEventRecord(c->ev_pool[slot].second, st);
    }
};

double taylor_poly_abs(int order, double y)
{
    std::complex<double> term(1.0, 0.0), sum(1.0, 0.0);
    const std::complex<double> iy(0.0, y);
    for (int k = 1; k <= order; ++k) {
        term *= iy / (double)k;
        sum += term;
    }
    return std::abs(sum);
}

// |sum_{k<=P} (-x)^k / k!|: the diffusion step's polynomial of exp(-x)
double taylor_real_poly_abs(int order, double x)
{
    double term = 1.0, sum = 1.0;
    for (int k = 1; k <= order; ++k) {
        term *= -x / (double)k;
        sum += term;
    }
    return std::fabs(sum);
}

}  // namespace

extern "C" double tdse_taylor_real_stability_limit(int32_t order)
{
    static std::mutex mu;
    static std::map<int, double> cache;
    if (order < 1 || order > 16) return 0.0;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(order);
    if (it != cache.end()) return it->second;
    const double tol = 1.0 + 1e-12;
    double x = 0.0;
    const double h = 1e-4;
    while (x < 20.0 && taylor_real_poly_abs(order, x + h) <= tol) x += h;
    double a = x, b = x + h;
    for (int i = 0; i < 60; ++i) {
        const double mid = 0.5 * (a + b);
        if (taylor_real_poly_abs(order, mid) <= tol) a = mid; else b = mid;
    }
    cache[order] = a;
    return a;
}

extern "C" double tdse_taylor_stability_limit(int32_t order)
{
    static std::mutex mu;
    static std::map<int, double> cache;
    if (order < 1 || order > 16) return 0.0;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(order);
    if (it != cache.end()) return it->second;
    // scan upward in small steps, then bisect the first crossing of 1 + 1e-12
    const double tol = 1.0 + 1e-12;
    double y = 0.0;
    const double h = 1e-4;
    while (y < 10.0 && taylor_poly_abs(order, y + h) <= tol) y += h;
    double a = y, b = y + h;
    for (int i = 0; i < 60; ++i) {
        const double mid = 0.5 * (a + b);
        if (taylor_poly_abs(order, mid) <= tol) a = mid; else b = mid;
    }
    cache[order] = a;
    return a;
}

// ---------------------------------------------------------------------------
// context creation
// ---------------------------------------------------------------------------
// Largest absolute row sum of H (eq. h_matrix) with the coupling scalar of
// the gauge bounded by e_max: |E| (length gauge: e_max r kappa per coupled
// row) or |A/c| (velocity gauge: e_max kappa (sum |first-derivative
// weights| + l/r) per coupled row).
static double gershgorin_bound(const tdse_grid_desc& g, double e_max, int gauge = 0)
{
    const double h2 = g.dr * g.dr;
    const double dk = (g.stencil == 3) ? 1.0 / h2 : 30.0 / (24.0 * h2);
    const double ok = (g.stencil == 3) ? 1.0 / h2 : 34.0 / (24.0 * h2);
    const double d1 = (g.stencil == 3) ? 1.0 / g.dr : 1.5 / g.dr;
    double best = 0.0;
    for (int l = 0; l <= g.lmax; ++l) {
        const double kl = (l > 0) ? std::sqrt((double)l * l / (4.0 * l * l - 1.0)) : 0.0;
        const double kp = (l < g.lmax) ? std::sqrt((double)(l + 1) * (l + 1) / (4.0 * (l + 1) * (l + 1) - 1.0)) : 0.0;
        for (int i = 0; i < g.n_r; ++i) {
            const double r = (double)(i + 1) * g.dr;
            const double d = dk + 0.5 * (double)l * (l + 1) / (r * r) - g.z_nuc / r;
            const double cpl = (gauge != 0) ? std::fabs(e_max) * (kl * (d1 + (double)l / r) + kp * (d1 + (double)(l + 1) / r))
                                            : std::fabs(e_max) * r * (kl + kp);
            best = std::max(best, std::fabs(d) + ok + cpl);
        }
    }
    return best;
}

static double cached_bound(const tdse_ctx* c, int k, double e_max)
{
    const std::tuple<int, int, double> key(k, c->gauge, std::fabs(e_max));
    auto it = c->bound_cache.find(key);
    if (it != c->bound_cache.end()) return it->second;
    const double b = gershgorin_bound(c->grids[k], std::fabs(e_max), c->gauge);
    c->bound_cache.emplace(key, b);
    return b;
}

// Bound on the coupling scalar of the gauge over a whole pulse (Sec. 3):
// length gauge |E| <= |E0| (sin^2 envelope on E) or |E0| (w + W) (on A/c,
// W = w / (2 n_c)); velocity gauge |A/c| <= |E0| (envelope on A/c) or
// 3 |E0| / w (on E: integrating sin^2(W tau) cos(w tau + phi) by parts
// leaves the envelope's value plus its total variation 2, over w).
static double coupling_bound(const tdse_ctx* c, const tdse_pulse& p)
{
    const double e = std::fabs(p.e0);
    if (c->gauge == 0) return (p.shape == 1) ? e * (p.omega + p.omega / (2.0 * p.n_cycles)) : e;
    return (p.shape == 1) ? e : 3.0 * e / p.omega;
}

static int states_for(int lmax)
{
    int s = 0;
    for (int l = 0; l <= std::min(lmax, 4); ++l) s += 5 - l;
    return s;
}

static int fused_width(int K, int stencil) { return kBlock - 2 * (K - 1) * (stencil == 3 ? 1 : 2); }
// output radii of one strip tile (kStripWaves strips of 64 - 2 K s)
static int strip_width(int K, int stencil) { return kStripWaves * (64 - 2 * K * (stencil == 3 ? 1 : 2)); }
// output radii of one pair-strip tile (two strips of 128 - 2 K s, two waves each)
static int pair_strip_width(int K, int stencil) { return kPairStrips * (128 - 2 * K * (stencil == 3 ? 1 : 2)); }

// (Re)builds one tile set.  rows = 0 for the population set.  The fused set
// (K = c->fuse_k terms per launch) uses radially overlapping tiles: tile t
// starts at radius t*W - (K-1)s and writes the W = 256 - 2(K-1)s radii
// [t*W, (t+1)*W).
static void build_tiles(tdse_ctx* c, int set, int rows)
{
    c->tiles[set].clear();
    if (set == kStripTiles || set == kRk4Tiles || set == kApplyTiles) {
        // tile r0 = first output radius; the kernel places its strips (the
        // RK4 strips are built for its four stages, the sweep strips for one)
        // (the sweep strips are aligned: 4 waves of 64 radii, no overlap)
        const int K = (set == kRk4Tiles) ? 4 : std::max(1, c->fuse_k);
        const int W = (set == kApplyTiles) ? kBlock
                      : (set == kStripTiles && c->fuse_kind >= 2) ? pair_strip_width(K, c->stencil)
                                                                  : strip_width(K, c->stencil);
        for (int k = 0; k < c->n_inst; ++k) {
            Inst& I = c->inst[k];
            I.tbegin[set] = (int32_t)c->tiles[set].size();
            for (int l0 = 0; l0 <= I.lmax; l0 += rows) {
                const int l1 = std::min(l0 + rows, I.lmax + 1);
                for (int o0 = 0; o0 < I.n; o0 += W) {
                    Tile t;
                    std::memset(&t, 0, sizeof t);
                    t.off = I.off;
                    t.tab_off = I.tab_off;
                    t.inst = k;
                    t.r0 = o0;
                    t.l0 = l0;
                    t.l1 = l1;
                    t.n = I.n;
                    t.lmax = I.lmax;
                    t.i_ion = I.i_ion;
                    t.n_states = I.n_states;
                    t.dr = I.dr;
                    t.inv_dr2 = I.inv_dr2;
                    t.z = I.z;
                    c->tiles[set].push_back(t);
                }
            }
            I.tend[set] = (int32_t)c->tiles[set].size();
        }
        if (set == kStripTiles) {
            // the persistent launch's order: the most rows first (a tile's
            // time grows with its rows), then the table order
            const std::vector<Tile>& T = c->tiles[set];
            c->strip_perm.resize(T.size());
            for (size_t i = 0; i < T.size(); ++i) c->strip_perm[i] = (int32_t)i;
            std::stable_sort(c->strip_perm.begin(), c->strip_perm.end(), [&](int32_t a, int32_t b) {
                return T[a].l1 - T[a].l0 > T[b].l1 - T[b].l0;
            });
        }
        return;
    }
    if (set == kFusedTiles) {
        const int K = std::max(1, c->fuse_k);
        const int s = (c->stencil == 3) ? 1 : 2;
        const int W = fused_width(K, c->stencil);
        for (int k = 0; k < c->n_inst; ++k) {
            Inst& I = c->inst[k];
            I.tbegin[set] = (int32_t)c->tiles[set].size();
            for (int l0 = 0; l0 <= I.lmax; l0 += rows) {
                for (int o0 = 0; o0 < I.n; o0 += W) {
                    Tile t;
                    std::memset(&t, 0, sizeof t);
                    t.off = I.off;
                    t.tab_off = I.tab_off;
                    t.inst = k;
                    t.r0 = o0 - (K - 1) * s;
                    t.l0 = l0;
                    t.l1 = std::min(l0 + rows, I.lmax + 1);
                    t.n = I.n;
                    t.lmax = I.lmax;
                    t.i_ion = I.i_ion;
                    t.n_states = I.n_states;
                    t.dr = I.dr;
                    t.inv_dr2 = I.inv_dr2;
                    t.z = I.z;
                    c->tiles[set].push_back(t);
                }
            }
            I.tend[set] = (int32_t)c->tiles[set].size();
        }
        return;
    }
    const int width = (set == kPairTiles) ? 2 * kBlock : kBlock;
    for (int k = 0; k < c->n_inst; ++k) {
        Inst& I = c->inst[k];
        I.tbegin[set] = (int32_t)c->tiles[set].size();
        const int lhi = (set == kPopTiles) ? std::min(I.lmax, 4) + 1 : I.lmax + 1;
        const int step = (set == kPopTiles) ? lhi : rows;
        for (int l0 = 0; l0 < lhi; l0 += step) {
            for (int r0 = 0; r0 < I.n; r0 += width) {
                Tile t;
                std::memset(&t, 0, sizeof t);
                t.off = I.off;
                t.tab_off = I.tab_off;
                t.inst = k;
                t.r0 = r0;
                t.l0 = l0;
                t.l1 = std::min(l0 + step, lhi);
                t.n = I.n;
                t.lmax = I.lmax;
                t.i_ion = I.i_ion;
                t.n_states = I.n_states;
                t.dr = I.dr;
                t.inv_dr2 = I.inv_dr2;
                t.z = I.z;
                c->tiles[set].push_back(t);
            }
        }
        I.tend[set] = (int32_t)c->tiles[set].size();
    }
}

// Tuning cache: a text file (path in TDSE_TUNE_CACHE) with one line per
// shape, "<key> <rows> <variant>", key = stencil.precision.log2(unknowns).log2(mean rows).
static std::string tune_key(const tdse_ctx* c)
{
    int64_t unknowns = 0, rows = 0;
    for (const tdse_grid_desc& g : c->grids) {
        unknowns += (int64_t)(g.lmax + 1) * g.n_r;
        rows += g.lmax + 1;
    }
    const int ub = (int)std::ceil(std::log2((double)std::max<int64_t>(unknowns, 1)));
    const int rb = (int)std::ceil(std::log2((double)std::max<int64_t>(rows / c->n_inst, 1)));
    return "s" + std::to_string(c->stencil) + ".p" + std::to_string(c->prec) + ".u" + std::to_string(ub) +
           ".l" + std::to_string(rb);
}

static int tune_cache_lookup(const tdse_ctx* c, int* variant)
{
    const char* path = std::getenv("TDSE_TUNE_CACHE");
    if (!path) return 0;
    FILE* f = std::fopen(path, "r");
    if (!f) return 0;
    const std::string key = tune_key(c);
    char kbuf[128];
    int rows = 0, var = 0, found = 0;
    while (std::fscanf(f, "%127s %d %d", kbuf, &rows, &var) == 3) {
        if (key == kbuf && rows >= 1 && rows <= kTileRows && var >= 0 && var <= 7) {
            found = rows;  // last entry wins
            *variant = var;
        }
    }
    std::fclose(f);
    return found;
}

static void tune_cache_store(const tdse_ctx* c, int rows, int variant)
{
    const char* path = std::getenv("TDSE_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d\n", tune_key(c).c_str(), rows, variant);
    std::fclose(f);
}

extern "C" tdse_status tdse_init_grid(const tdse_grid_desc* grids, int32_t n_inst, tdse_ctx** out)
{
    if (!out) return TDSE_E_INVALID;
    *out = nullptr;
    if (!grids || n_inst < 1 || n_inst > (1 << 20)) return TDSE_E_INVALID;
    tdse_ctx* c = new (std::nothrow) tdse_ctx;
    if (!c) return TDSE_E_NOMEM;
    c->n_inst = n_inst;
    c->grids.assign(grids, grids + n_inst);
    c->stencil = grids[0].stencil;
    c->prec = grids[0].precision;
    for (int k = 0; k < n_inst; ++k) {
        const tdse_grid_desc& g = grids[k];
        if (g.n_r < 8 || g.n_r > (1 << 26) || g.lmax < 0 || g.lmax > 1023 ||
            (g.stencil != 3 && g.stencil != 5) || (g.precision != TDSE_FP64 && g.precision != TDSE_FP32 && g.precision != TDSE_FP48) ||
            !(g.dr > 0.0) || !(g.z_nuc > 0.0) || !std::isfinite(g.r_ion) || g.stencil != c->stencil ||
            g.precision != c->prec) {
            delete c;
            return TDSE_E_INVALID;
        }
    }
    c->elem = (c->prec == TDSE_FP64) ? 16 : (c->prec == TDSE_FP48) ? 12 : 8;
    // instance table, offsets aligned to 64 elements
    int lmax_all = 0;
    int64_t off = 0, tab = 0;
    c->inst.resize(n_inst);
    for (int k = 0; k < n_inst; ++k) {
        const tdse_grid_desc& g = grids[k];
        Inst& I = c->inst[k];
        std::memset(&I, 0, sizeof I);
        I.off = off;
        I.n = g.n_r;
        I.lmax = g.lmax;
        I.n_states = states_for(g.lmax);
        I.dr = g.dr;
        I.inv_dr2 = 1.0 / (g.dr * g.dr);
        I.z = g.z_nuc;
        int i_ion = 0;
        while (i_ion < g.n_r && (double)(i_ion + 1) * g.dr <= g.r_ion) ++i_ion;
        I.i_ion = i_ion;
        I.tab_off = tab;
        I.breakdown = 1e-12 * gershgorin_bound(g, 0.0, 0);
        I.i_flux = -1;
        tab += (int64_t)(1 + I.n_states) * g.n_r;
        off += ((int64_t)(g.lmax + 1) * g.n_r + 63) / 64 * 64;
        lmax_all = std::max(lmax_all, g.lmax);
    }
    c->state_elems = off;
    c->kappa.resize(lmax_all + 2);
    for (int l = 0; l < lmax_all + 2; ++l)
        c->kappa[l] = (l > 0) ? std::sqrt((double)l * l / (4.0 * l * l - 1.0)) : 0.0;

    // Tile sets.  Sweeps: rows per tile from the tuning cache if it has this
    // shape, else chosen so the launch has >= kTargetTiles workgroups.
    // Reductions (Lanczos, copies): up to 16 rows, >= 1024 workgroups.
    // Populations: one tile per 256 radial points covering rows 0..min(lmax, 4).
    int64_t total_cols = 0;
    for (int k = 0; k < n_inst; ++k)
        total_cols += (int64_t)((grids[k].n_r + kBlock - 1) / kBlock) * (grids[k].lmax + 1);
    c->total_cols = total_cols;
    int rows = kTileRows;
    while (rows > 1 && total_cols / rows < kTargetTiles) rows /= 2;
    int cached_variant = 0;
    const int cached = tune_cache_lookup(c, &cached_variant);
    c->rows_sweep = cached > 0 ? cached : rows;
    c->sweep_variant = cached > 0 ? cached_variant : 0;
    int rr = 16;
    while (rr > 1 && total_cols / rr < 1024) rr /= 2;
    c->rows_reduce = rr;
    build_tiles(c, kSweepTiles, c->rows_sweep);
    build_tiles(c, kReduceTiles, c->rows_reduce);
    // observables: up to kObsRows rows (a thread loads all of its rows at
    // once), >= 256 workgroups; taller tiles leave fewer partial sums to finish
    int ro = kObsRows;
    while (ro > 1 && total_cols / ro < 256) ro /= 2;
    c->rows_obs = ro;
    // RK4 strips: up to 16 rows, >= 1024 workgroups where the grid allows
    int64_t rk4_cols = 0;
    for (int k = 0; k < n_inst; ++k)
        rk4_cols += (int64_t)((grids[k].n_r + strip_width(4, c->stencil) - 1) / strip_width(4, c->stencil)) *
                    (grids[k].lmax + 1);
    int r4 = 16;
    while (r4 > 1 && rk4_cols / r4 < 1024) r4 /= 2;
    c->rows_rk4 = r4;
    build_tiles(c, kObsTiles, c->rows_obs);
    build_tiles(c, kPopTiles, 0);
    build_tiles(c, kFusedTiles, c->rows_fused);
    build_tiles(c, kPairTiles, c->rows_sweep);
    build_tiles(c, kStripTiles, c->rows_fused);
    build_tiles(c, kRk4Tiles, c->rows_rk4);
    build_tiles(c, kApplyTiles, c->rows_sweep);
    // radial tables: u0 (normalised r exp(-z r)) and the bound eigenvectors
    c->radial.assign(tab, 0.0);
    std::vector<std::thread> pool;
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<int> next(1, 0);
    std::mutex mu;
    auto worker = [&]() {
        for (;;) {
            int k;
            {
                std::lock_guard<std::mutex> lock(mu);
                if (next[0] >= n_inst) return;
                k = next[0]++;
            }
            const tdse_grid_desc& g = grids[k];
            const Inst& I = c->inst[k];
            double* t = c->radial.data() + I.tab_off;
            double s = 0.0;
            for (int i = 0; i < g.n_r; ++i) {
                const double r = (double)(i + 1) * g.dr;
                t[i] = r * std::exp(-g.z_nuc * r);
                s += t[i] * t[i];
            }
            const double nrm = 1.0 / std::sqrt(g.dr * s);
            for (int i = 0; i < g.n_r; ++i) t[i] *= nrm;
            int row = 1;
            for (int l = 0; l <= std::min(g.lmax, 4); ++l) {
                std::vector<double> e, v;
                lowest_radial_states(g.n_r, g.stencil, g.dr, g.z_nuc, l, 5 - l, e, v);
                std::memcpy(t + (size_t)row * g.n_r, v.data(), v.size() * sizeof(double));
                row += 5 - l;
            }
        }
    };
    for (unsigned w = 0; w < std::min<unsigned>(hw, (unsigned)n_inst); ++w) pool.emplace_back(worker);
    for (auto& th : pool) th.join();

    // workspace layout
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, kAlign);
        return at;
    };
    c->off_inst = take(sizeof(Inst) * n_inst);
    for (int set = 0; set < kNumTileSets; ++set) {
        // the sweep and fused sets may be rebuilt by the autotuners: room for
        // one row per tile (and, fused, the narrowest tile width)
        size_t cap = c->tiles[set].size();
        if (set == kSweepTiles) cap = (size_t)c->total_cols;
        if (set == kStripTiles || set == kRk4Tiles || set == kApplyTiles) {
            cap = 0;
            // the narrowest tiles either strip kernel builds
            const int W = std::min(strip_width(kMaxFused, c->stencil), pair_strip_width(kMaxFused, c->stencil));
            for (const tdse_grid_desc& g : c->grids) cap += (size_t)((g.n_r + W - 1) / W) * (g.lmax + 1);
            if (set == kStripTiles) c->strip_units_cap = cap * kStripWaves;
        }
        if (set == kPairTiles) {
            cap = 0;
            for (const tdse_grid_desc& g : c->grids) cap += (size_t)((g.n_r + 2 * kBlock - 1) / (2 * kBlock)) * (g.lmax + 1);
        }
        if (set == kFusedTiles) {
            cap = 0;
            const int W = fused_width(kMaxFused, c->stencil);
            for (const tdse_grid_desc& g : c->grids) cap += (size_t)((g.n_r + W - 1) / W) * (g.lmax + 1);
        }
        c->tile_cap[set] = cap;
        c->off_tiles[set] = take(sizeof(Tile) * cap);
    }
    c->off_kappa = take(sizeof(double) * c->kappa.size());
    // one all-zero row (the longest N, FP64 complex): the strip kernel reads
    // rows outside [0, lmax] from it
    int max_n = 0;
    for (const tdse_grid_desc& g : c->grids) max_n = std::max(max_n, g.n_r);
    c->zero_bytes = (size_t)max_n * 16;
    c->off_zero = take(c->zero_bytes);
    c->off_radial = take(sizeof(double) * c->radial.size());
    c->off_step = take(sizeof(double) * kSlots * (size_t)n_inst * kEtabSteps);
    c->off_obs_tmp = take(sizeof(tdse_obs) * n_inst);
    c->off_lz = take(sizeof(LanczosScalars) * n_inst);
    c->off_flux = take(sizeof(double) * 2 * (size_t)n_inst);
    c->off_queue = take(sizeof(unsigned) * 2);
    c->off_perm = take(sizeof(int32_t) * c->tile_cap[kStripTiles]);
    // Lanczos dots; the observables pass; or the strips' main partials (two
    // sets, by step parity) and the population tiles
    // (and the Runge-Kutta stages' deviation partials, one per sweep tile:
    // at most total_cols, the one-row tiling)
    c->partial_doubles = std::max({(size_t)c->total_cols, (size_t)c->tiles[kReduceTiles].size() * 2 * kMaxKrylov,
                                   (size_t)c->tiles[kObsTiles].size() * kObsMainQ +
                                       (size_t)c->tiles[kPopTiles].size() * kObsPopQ,
                                   2 * c->strip_units_cap * kObsMainQ +
                                       (size_t)c->tiles[kPopTiles].size() * kObsPopQ});
    c->off_partial = take(sizeof(double) * c->partial_doubles);
    c->off_vecs = o;
    c->fixed_bytes = o;
    *out = c;
    return TDSE_OK;
}

extern "C" void tdse_destroy(tdse_ctx* c)
{
    if (!c) return;
    c->drop_graphs();
    if (c->obs_stream) {
        (void)hipStreamSynchronize(c->obs_stream);
        (void)hipStreamDestroy(c->obs_stream);
        for (hipEvent_t ev : {c->obs_fork, c->obs_join, c->obs_done[0], c->obs_done[1]}) (void)hipEventDestroy(ev);
    }
    for (auto& e : c->ev_pool) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (int b = 0; b < 2; ++b) {
        if (c->step_ev[b]) {
            (void)hipEventSynchronize(c->step_ev[b]);
            (void)hipEventDestroy(c->step_ev[b]);
        }
        if (c->h_step[b]) (void)hipHostFree(c->h_step[b]);
    }
    delete c;
}

extern "C" const char* tdse_last_error(const tdse_ctx* c) { return c ? c->err.c_str() : "null context"; }
extern "C" int32_t tdse_num_instances(const tdse_ctx* c) { return c ? c->n_inst : 0; }
extern "C" int64_t tdse_state_offset(const tdse_ctx* c, int32_t k)
{
    return (c && k >= 0 && k < c->n_inst) ? c->inst[k].off : -1;
}
extern "C" size_t tdse_state_bytes(const tdse_ctx* c) { return c ? c->state_bytes() : 0; }
extern "C" size_t tdse_workspace_bytes(const tdse_ctx* c, int32_t method, int32_t order_or_m)
{
    if (!c) return 0;
    return c->fixed_bytes + c->vecs_needed(method, order_or_m) * c->state_bytes();
}

extern "C" double tdse_lambda_max_bound(const tdse_ctx* c, int32_t k, double e_max)
{
    if (!c || k < 0 || k >= c->n_inst) return -1.0;
    return cached_bound(c, k, e_max);
}

// ---------------------------------------------------------------------------
// binding and state transfer
// ---------------------------------------------------------------------------
extern "C" tdse_status tdse_bind(tdse_ctx* c, void* d_state, void* d_work, size_t work_bytes,
                                 void* hip_stream)
{
    if (!c) return TDSE_E_INVALID;
    if (!d_state || !d_work) return c->fail(TDSE_E_INVALID, "tdse_bind: null device pointer");
    if ((reinterpret_cast<uintptr_t>(d_state) | reinterpret_cast<uintptr_t>(d_work)) % kAlign)
        return c->fail(TDSE_E_INVALID, "tdse_bind: device buffers must be 256-byte aligned");
    if (work_bytes < c->fixed_bytes)
        return c->fail(TDSE_E_WORKSPACE, "tdse_bind: workspace smaller than the fixed tables");
    c->drop_graphs();
    c->lz_m = 0;
    c->d_state = static_cast<char*>(d_state);
    c->d_work = static_cast<char*>(d_work);
    c->work_bytes = work_bytes;
    c->stream = static_cast<hipStream_t>(hip_stream);
    for (int b = 0; b < 2; ++b) {
        if (!c->h_step[b]) {
            hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&c->h_step[b]),
                                         sizeof(double) * kSlots * (size_t)c->n_inst * kEtabSteps);
            if (e != hipSuccess) return c->hip_fail(e, "hipHostMalloc");
            e = hipEventCreateWithFlags(&c->step_ev[b], hipEventDisableTiming);
            if (e != hipSuccess) return c->hip_fail(e, "hipEventCreate");
        }
    }
    struct Up {
        size_t off;
        const void* src;
        size_t bytes;
    } ups[] = {
        {c->off_inst, c->inst.data(), sizeof(Inst) * c->inst.size()},
        {c->off_tiles[kSweepTiles], c->tiles[kSweepTiles].data(), sizeof(Tile) * c->tiles[kSweepTiles].size()},
        {c->off_tiles[kReduceTiles], c->tiles[kReduceTiles].data(), sizeof(Tile) * c->tiles[kReduceTiles].size()},
        {c->off_tiles[kObsTiles], c->tiles[kObsTiles].data(), sizeof(Tile) * c->tiles[kObsTiles].size()},
        {c->off_tiles[kPopTiles], c->tiles[kPopTiles].data(), sizeof(Tile) * c->tiles[kPopTiles].size()},
        {c->off_tiles[kFusedTiles], c->tiles[kFusedTiles].data(), sizeof(Tile) * c->tiles[kFusedTiles].size()},
        {c->off_tiles[kPairTiles], c->tiles[kPairTiles].data(), sizeof(Tile) * c->tiles[kPairTiles].size()},
        {c->off_tiles[kStripTiles], c->tiles[kStripTiles].data(), sizeof(Tile) * c->tiles[kStripTiles].size()},
        {c->off_tiles[kRk4Tiles], c->tiles[kRk4Tiles].data(), sizeof(Tile) * c->tiles[kRk4Tiles].size()},
        {c->off_tiles[kApplyTiles], c->tiles[kApplyTiles].data(), sizeof(Tile) * c->tiles[kApplyTiles].size()},
        {c->off_kappa, c->kappa.data(), sizeof(double) * c->kappa.size()},
        {c->off_radial, c->radial.data(), sizeof(double) * c->radial.size()},
        {c->off_perm, c->strip_perm.data(), sizeof(int32_t) * c->strip_perm.size()},
    };
    for (const Up& u : ups) {
        hipError_t e = hipMemcpyAsync(c->d_work + u.off, u.src, u.bytes, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "tdse_bind upload");
    }
    hipError_t e = hipMemsetAsync(c->d_work + c->off_zero, 0, c->zero_bytes, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "tdse_bind zero row");
    e = hipMemsetAsync(c->d_work + c->off_flux, 0, sizeof(double) * 2 * (size_t)c->n_inst, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "tdse_bind flux");
    // the work queue's counters start at zero (each persistent launch leaves them so)
    e = hipMemsetAsync(c->d_queue(), 0, sizeof(unsigned) * 2, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "tdse_bind queue");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "tdse_bind sync");
    c->bound = true;
    return TDSE_OK;
}

extern "C" tdse_status tdse_set_state(tdse_ctx* c, int32_t k, const double* host)
{
    if (!c) return TDSE_E_INVALID;
    if (!c->bound) return c->fail(TDSE_E_UNBOUND, "tdse_set_state: not bound");
    if (k < 0 || k >= c->n_inst) return c->fail(TDSE_E_INVALID, "tdse_set_state: bad instance");
    const Inst& I = c->inst[k];
    const size_t cnt = (size_t)(I.lmax + 1) * I.n;
    std::vector<double> tmp;
    if (!host) {
        tmp.assign(2 * cnt, 0.0);
        for (int i = 0; i < I.n; ++i) tmp[2 * i] = c->radial[I.tab_off + i];
        host = tmp.data();
    }
    hipError_t e;
    char* dst = c->d_state + (size_t)I.off * c->elem;
    if (c->prec == TDSE_FP64) {
        e = hipMemcpyAsync(dst, host, cnt * 16, hipMemcpyHostToDevice, c->stream);
    } else if (c->prec == TDSE_FP48) {
        // plane h: upper words of (re, im); plane l: the next 16 bits of
        // each, rounded to nearest (ties away from zero) as the kernels store
        std::vector<uint32_t> h(2 * cnt), l(cnt);
        for (size_t j = 0; j < cnt; ++j) {
            uint64_t a, b;
            std::memcpy(&a, host + 2 * j, 8);
            std::memcpy(&b, host + 2 * j + 1, 8);
            a += 0x8000u;
            b += 0x8000u;
            h[2 * j] = (uint32_t)(a >> 32);
            h[2 * j + 1] = (uint32_t)(b >> 32);
            l[j] = ((uint32_t)a >> 16) | ((uint32_t)b & 0xffff0000u);
        }
        char* dl = c->d_state + 8 * (size_t)c->plane() + 4 * (size_t)I.off;
        e = hipMemcpyAsync(c->d_state + 8 * (size_t)I.off, h.data(), cnt * 8, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(dl, l.data(), cnt * 4, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    } else {
        std::vector<float> f(2 * cnt);
        for (size_t j = 0; j < 2 * cnt; ++j) f[j] = (float)host[j];
        e = hipMemcpyAsync(dst, f.data(), cnt * 8, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return (e == hipSuccess) ? TDSE_OK : c->hip_fail(e, "tdse_set_state");
}

extern "C" tdse_status tdse_get_state(tdse_ctx* c, int32_t k, double* host)
{
    if (!c || !host) return TDSE_E_INVALID;
    if (!c->bound) return c->fail(TDSE_E_UNBOUND, "tdse_get_state: not bound");
    if (k < 0 || k >= c->n_inst) return c->fail(TDSE_E_INVALID, "tdse_get_state: bad instance");
    const Inst& I = c->inst[k];
    const size_t cnt = (size_t)(I.lmax + 1) * I.n;
    const char* src = c->d_state + (size_t)I.off * c->elem;
    hipError_t e;
    if (c->prec == TDSE_FP64) {
        e = hipMemcpyAsync(host, src, cnt * 16, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    } else if (c->prec == TDSE_FP48) {
        std::vector<uint32_t> h(2 * cnt), l(cnt);
        e = hipMemcpyAsync(h.data(), c->d_state + 8 * (size_t)I.off, cnt * 8, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(l.data(), c->d_state + 8 * (size_t)c->plane() + 4 * (size_t)I.off, cnt * 4,
                               hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        for (size_t j = 0; j < cnt; ++j) {
            const uint64_t a = ((uint64_t)h[2 * j] << 32) | (uint64_t)(l[j] << 16);
            const uint64_t b = ((uint64_t)h[2 * j + 1] << 32) | (uint64_t)(l[j] & 0xffff0000u);
            std::memcpy(host + 2 * j, &a, 8);
            std::memcpy(host + 2 * j + 1, &b, 8);
        }
    } else {
        std::vector<float> f(2 * cnt);
        e = hipMemcpyAsync(f.data(), src, cnt * 8, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        for (size_t j = 0; j < 2 * cnt; ++j) host[j] = (double)f[j];
    }
    return (e == hipSuccess) ? TDSE_OK : c->hip_fail(e, "tdse_get_state");
}

// ---------------------------------------------------------------------------
// per-step scalars
// ---------------------------------------------------------------------------
namespace {

double field_at(const tdse_pulse& p, double t)
{
    const double tau = t - p.t_on;
    const double period = 2.0 * M_PI * p.n_cycles / p.omega;
    if (!(tau >= 0.0 && tau <= period)) return 0.0;
    const double s = std::sin(M_PI * tau / period);
    if (p.shape == 1) {
        // sin^2 envelope on A/c = -E0 sin^2(W tau) sin(w tau + phi), W = pi / T:
        // E = -d(A/c)/dt
        const double w_env = M_PI / period;
        const double cs = std::cos(M_PI * tau / period);
        return p.e0 * s * (p.omega * s * std::cos(p.omega * tau + p.cep) +
                           2.0 * w_env * cs * std::sin(p.omega * tau + p.cep));
    }
    return p.e0 * s * s * std::cos(p.omega * tau + p.cep);
}

// Sec. 3, eq. VectorStep with A/c in place of A: the change of A/c over
// [t, t + h], -int E, by the 5-point Gauss-Legendre rule (the roots 0,
// +-sqrt(5 -+ 2 sqrt(10/7)) / 3 of the Legendre polynomial P_5, weights
// 128/225 and (322 +- 13 sqrt(70)) / 900), nodes taken in increasing order.
double vp_increment(const tdse_pulse& p, double t, double h)
{
    const double xa = std::sqrt(5.0 - 2.0 * std::sqrt(10.0 / 7.0)) / 3.0;
    const double xb = std::sqrt(5.0 + 2.0 * std::sqrt(10.0 / 7.0)) / 3.0;
    const double wa = (322.0 + 13.0 * std::sqrt(70.0)) / 900.0;
    const double wb = (322.0 - 13.0 * std::sqrt(70.0)) / 900.0;
    const double x[5] = {-xb, -xa, 0.0, xa, xb};
    const double w[5] = {wb, wa, 128.0 / 225.0, wa, wb};
    double sum = 0.0;
    for (int j = 0; j < 5; ++j) sum += w[j] * field_at(p, t + 0.5 * h * (1.0 + x[j]));
    return -0.5 * h * sum;
}

// A/c at t0, -int_{t_on}^{t0} E, by the same rule over ceil((t0 - t_on) / dt)
// equal pieces in time order (the increments of steps of dt from t_on).
double vp_at(const tdse_pulse& p, double t0, double dt)
{
    if (!(t0 > p.t_on)) return 0.0;
    const double span = t0 - p.t_on;
    int64_t m = (int64_t)std::ceil(span / dt - 1e-9);
    if (m < 1) m = 1;
    const double piece = span / (double)m;
    double a = 0.0;
    for (int64_t q = 0; q < m; ++q) a += vp_increment(p, p.t_on + (double)q * piece, piece);
    return a;
}

// Fills and uploads the scalars of steps [s0, s0 + count) (count <= kEtabSteps)
// for every instance; returns the device base of the chunk.
tdse_status upload_steps(tdse_ctx* c, const tdse_pulse* pulses, const double* t0, const double* dt,
                         int64_t s0, int count, int obs_every)
{
    const int b = c->step_buf;
    c->step_buf ^= 1;
    if (c->step_ev_used[b]) {
        hipError_t e = hipEventSynchronize(c->step_ev[b]);
        if (e != hipSuccess) return c->hip_fail(e, "step staging wait");
    }
    double* h = c->h_step[b];
    const int n = c->n_inst;
    const bool vel = c->gauge != 0 && pulses != nullptr;
    if (vel && s0 == 0) {
        c->a_run.assign(n, 0.0);
        for (int k = 0; k < n; ++k) c->a_run[k] = vp_at(pulses[k], t0[k], dt[k]);
    }
    for (int s = 0; s < count; ++s) {
        double* row = h + (size_t)s * kSlots * n;
        for (int k = 0; k < n; ++k) {
            const double step = (double)(s0 + s);
            const double ts = t0[k] + step * dt[k];
            const double tm = t0[k] + (step + 0.5) * dt[k];
            const double te = t0[k] + (step + 1.0) * dt[k];
            const double e_end = pulses ? field_at(pulses[k], te) : 0.0;
            if (vel) {
                // A/c at the stage times: A/c(t_n) plus the quadrature from t_n
                const tdse_pulse& p = pulses[k];
                const double a = c->a_run[k];
                row[kEStart * n + k] = a + vp_increment(p, ts, 0.0 * dt[k]);
                row[kEMid * n + k] = a + vp_increment(p, ts, 0.5 * dt[k]);
                row[kEEnd * n + k] = a + vp_increment(p, ts, 1.0 * dt[k]);
                for (int i = 0; i < kRkMax; ++i)
                    row[(kEStage0 + i) * n + k] = (i < c->rk_stages) ? a + vp_increment(p, ts, c->rk_c[i] * dt[k]) : 0.0;
                c->a_run[k] = a + vp_increment(p, ts, dt[k]);
            } else {
                row[kEStart * n + k] = pulses ? field_at(pulses[k], ts) : 0.0;
                row[kEMid * n + k] = pulses ? field_at(pulses[k], tm) : 0.0;
                row[kEEnd * n + k] = e_end;
                for (int i = 0; i < kRkMax; ++i)
                    row[(kEStage0 + i) * n + k] =
                        (pulses && i < c->rk_stages) ? field_at(pulses[k], t0[k] + (step + c->rk_c[i]) * dt[k]) : 0.0;
            }
            row[kEObs * n + k] = e_end;
            row[kTEnd * n + k] = te;
            row[kDt * n + k] = dt[k];
            const int64_t done = s0 + s + 1;
            row[kRec * n + k] = (obs_every > 0 && done % obs_every == 0) ? (double)(done / obs_every - 1) : -1.0;
        }
    }
    hipError_t e = hipMemcpyAsync(c->d_step(), h, sizeof(double) * kSlots * n * (size_t)count,
                                  hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "step upload");
    e = hipEventRecord(c->step_ev[b], c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "step event");
    c->step_ev_used[b] = true;
    return TDSE_OK;
}

tdse_status check_common(tdse_ctx* c, const tdse_pulse* pulses, const double* t0, const double* dt,
                         int32_t nsteps, int32_t obs_every, tdse_obs* d_obs, int method, int order)
{
    if (!c->bound) return c->fail(TDSE_E_UNBOUND, "step: no device memory bound");
    if (!pulses || !t0 || !dt) return c->fail(TDSE_E_INVALID, "step: null argument");
    if (nsteps < 0) return c->fail(TDSE_E_INVALID, "step: nsteps < 0");
    if (obs_every < 0) return c->fail(TDSE_E_INVALID, "step: obs_every < 0");
    if (obs_every > 0 && !d_obs) return c->fail(TDSE_E_INVALID, "step: observables requested, d_obs is null");
    for (int k = 0; k < c->n_inst; ++k) {
        if (!std::isfinite(t0[k]) || !(dt[k] > 0.0) || !std::isfinite(dt[k]))
            return c->fail(TDSE_E_INVALID, "step: t0 must be finite and dt > 0");
        if (!(pulses[k].omega > 0.0) || !(pulses[k].n_cycles > 0.0) || !std::isfinite(pulses[k].e0))
            return c->fail(TDSE_E_INVALID, "step: pulse needs omega > 0, n_cycles > 0, finite e0");
        if (pulses[k].shape != TDSE_PULSE_SINE2_E && pulses[k].shape != TDSE_PULSE_SINE2_A)
            return c->fail(TDSE_E_INVALID, "step: unknown pulse shape");
    }
    const size_t need = tdse_workspace_bytes(c, method, order);
    if (c->work_bytes < need)
        return c->fail(TDSE_E_WORKSPACE, "step: workspace too small for this method (" +
                                             std::to_string(need) + " bytes needed)");
    return TDSE_OK;
}

tdse_status check_stable(tdse_ctx* c, const tdse_pulse* pulses, const double* dt, int order)
{
    const double y = tdse_taylor_stability_limit(order);
    for (int k = 0; k < c->n_inst; ++k) {
        const double lam = cached_bound(c, k, coupling_bound(c, pulses[k]));
        if (dt[k] * lam > y) {
            char buf[256];
            std::snprintf(buf, sizeof buf,
                          "instance %d: dt*lambda_max = %.4g exceeds the order-%d stability limit %.4g "
                          "(dt must be <= %.4g)", k, dt[k] * lam, order, y, y / lam);
            return c->fail(TDSE_E_UNSTABLE, buf);
        }
    }
    return TDSE_OK;
}

// observables of the state after step s (within the uploaded chunk at `step`)
hipError_t launch_obs(tdse_ctx* c, const void* psi, const double* step, double* records,
                      int64_t rec_stride, hipStream_t st, double* partial = nullptr)
{
    TimedLaunch tl(c, 2, st);
    const SweepGeom red = c->geom(kObsTiles), pop = c->geom(kPopTiles);
    double* pmain = partial ? partial : c->d_partial();
    double* ppop = pmain + (size_t)red.n_tiles * kObsMainQ;
    hipError_t e = launch_obs_partial(c->prec, red, pop, c->d_radial(), psi, pmain, ppop, st);
    if (e != hipSuccess) return e;
    return launch_obs_finish(red, pop, pmain, ppop, step, rec_stride, records, st);
}

// observables of the state after a step whose last launch (Horner strips)
// wrote the main partial sums to pstrip: the population tiles, then the
// finish over the strips
static hipError_t launch_obs_strips(tdse_ctx* c, const void* psi, const double* pstrip, const double* step,
                                    double* records, int64_t rec_stride, hipStream_t st)
{
    TimedLaunch tl(c, 2, st);
    SweepGeom red = c->geom(kObsTiles), pop = c->geom(kPopTiles);
    red.n_tiles = 0;   // population tiles only
    double* ppop = c->d_partial() + 2 * c->strip_units_cap * kObsMainQ;
    hipError_t e = launch_obs_partial(c->prec, red, pop, c->d_radial(), psi, nullptr, ppop, st);
    if (e != hipSuccess) return e;
    return launch_obs_finish(red, pop, pstrip, ppop, step, rec_stride, records, st, kStripTiles, kStripWaves,
                             (int64_t)c->tiles[kStripTiles].size() * kStripWaves);
}

static hipError_t ensure_obs_stream(tdse_ctx* c)
{
    if (c->obs_stream) return hipSuccess;
    hipError_t e = hipStreamCreateWithFlags(&c->obs_stream, hipStreamNonBlocking);
    for (hipEvent_t* ev : {&c->obs_fork, &c->obs_join, &c->obs_done[0], &c->obs_done[1]})
        if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    return e;
}

// Enqueues the launches of steps [s0, s0 + count) of the current chunk.
// *cur is the buffer holding psi (the state, or the ping-pong vector of the
// fused Taylor path); a step function may move it.
//
// side: the observables of step s run on the second stream, concurrently with
// step s+1.  This needs a step function that never writes the buffer holding
// psi at its start (the Taylor rotation: psi(s) is overwritten first in step
// s+2).  Step s+2 waits for the observables of step s; the
// second stream runs them in order (they share the partial-sum buffer) and
// rejoins the main stream at the end of the chunk, so a chunk (and its
// captured graph) leaves nothing running on it.
//
// hooks: after each step, the absorbing mask (in place on psi; the
// observables then run their own pass) and the flux yield, where set.
template <typename StepFn>
hipError_t enqueue_chunk(tdse_ctx* c, int64_t s0, int count, int32_t obs_every, tdse_obs* d_obs,
                         int64_t rec_stride, void** cur, StepFn& step_fn, bool side, bool hooks)
{
    const bool absorb = hooks && c->absorber_on;
    const bool flux = hooks && c->flux_on;
    auto obs_at = [&](int s) { return obs_every > 0 && s >= 0 && (s0 + s + 1) % obs_every == 0; };
    bool forked = false;
    for (int s = 0; s < count; ++s) {
        const double* step = c->d_step() + (size_t)s * kSlots * c->n_inst;
        hipError_t e = hipSuccess;
        if (side && obs_at(s - 2)) e = hipStreamWaitEvent(c->stream, c->obs_done[s & 1], 0);
        // a step function that can sum the main observables in its last
        // launch does so into the partial set of this step's parity (the
        // step two later, which reuses it, waits for these observables)
        double* pstrip = c->d_partial() + (size_t)(s & 1) * c->strip_units_cap * kObsMainQ;
        c->obs_req = (c->obs_fusion && !absorb && obs_at(s)) ? pstrip : nullptr;
        c->obs_main_done = false;
        if (e == hipSuccess) e = step_fn(step);
        c->obs_req = nullptr;
        if (e == hipSuccess && absorb) e = launch_mask(c->prec, c->geom(kReduceTiles), *cur, c->stream);
        if (e == hipSuccess && flux)
            e = launch_flux(c->prec, c->stencil == 3 ? 1 : 2, c->geom(kReduceTiles), *cur, step, 0, c->d_jprev(),
                            c->d_yield(), c->stream);
        if (e != hipSuccess) return e;
        if (!obs_at(s)) continue;
        const bool fused = c->obs_main_done;
        auto obs_launch = [&](hipStream_t st) {
            return fused ? launch_obs_strips(c, *cur, pstrip, step, reinterpret_cast<double*>(d_obs), rec_stride, st)
                         : launch_obs(c, *cur, step, reinterpret_cast<double*>(d_obs), rec_stride, st);
        };
        if (!side) {
            e = obs_launch(c->stream);
        } else {
            e = hipEventRecord(c->obs_fork, c->stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(c->obs_stream, c->obs_fork, 0);
            if (e == hipSuccess) e = obs_launch(c->obs_stream);
            if (e == hipSuccess) e = hipEventRecord(c->obs_done[s & 1], c->obs_stream);
            forked = true;
        }
        if (e != hipSuccess) return e;
    }
    if (forked) {
        hipError_t e = hipEventRecord(c->obs_join, c->obs_stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->obs_join, 0);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Runs nsteps steps in chunks of kEtabSteps.  With graphs on (and timing
// off), the launches of a chunk are captured once into a hipGraph and the
// executable graph is replayed for every chunk with the same pattern; the
// per-step scalars (fields, times, record indices) are uploaded before each
// chunk, so the graph itself never changes.
template <typename StepFn>
tdse_status run_steps(tdse_ctx* c, const tdse_pulse* pulses, const double* t0, const double* dt,
                      int32_t nsteps, int32_t obs_every, tdse_obs* d_obs, int64_t method_key,
                      void** cur, StepFn&& step_fn, bool obs_side_ok = false)
{
    const int64_t n_rec = (obs_every > 0) ? nsteps / obs_every : 0;
    const int64_t rec_stride = n_rec * (int64_t)kObsRecord;
    const bool graphs = c->use_graphs && !c->timing && c->stream != nullptr;
    const bool side = obs_side_ok && obs_every > 0 && c->obs_overlap;
    if (side) {
        hipError_t e = ensure_obs_stream(c);
        if (e != hipSuccess) return c->hip_fail(e, "observables stream");
    }
    for (int64_t s0 = 0; s0 < nsteps; s0 += kEtabSteps) {
        const int count = (int)std::min<int64_t>(kEtabSteps, nsteps - s0);
        tdse_status st = upload_steps(c, pulses, t0, dt, s0, count, obs_every);
        if (st != TDSE_OK) return st;
        if (c->flux_on && s0 == 0) {
            // the current of the state the steps start from (the trapezoid's
            // first point; the velocity gauge takes A/c at the first step's start)
            hipError_t e = launch_flux(c->prec, c->stencil == 3 ? 1 : 2, c->geom(kReduceTiles), *cur, c->d_step(), 1,
                                       c->d_jprev(), c->d_yield(), c->stream);
            if (e != hipSuccess) return c->hip_fail(e, "flux start");
        }
        if (!graphs) {
            hipError_t e = enqueue_chunk(c, s0, count, obs_every, d_obs, rec_stride, cur, step_fn, side, true);
            if (e != hipSuccess) return c->hip_fail(e, "step launch");
            continue;
        }
        void* cur_start = *cur;
        const std::vector<int64_t> key = {method_key, count, obs_every,
                                          obs_every > 0 ? s0 % obs_every : 0,
                                          (int64_t)reinterpret_cast<uintptr_t>(d_obs), rec_stride,
                                          (int64_t)reinterpret_cast<uintptr_t>(cur_start),
                                          (c->absorber_on ? 1 : 0) + (c->flux_on ? 2 : 0)};
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return c->hip_fail(e, "hipStreamBeginCapture");
            hipError_t el = enqueue_chunk(c, s0, count, obs_every, d_obs, rec_stride, cur, step_fn, side, true);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(c->stream, &graph);
            if (el != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return c->hip_fail(el, "step launch during capture");
            }
            if (e != hipSuccess) return c->hip_fail(e, "hipStreamEndCapture");
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return c->hip_fail(e, "hipGraphInstantiate");
            it = c->graphs.emplace(key, exec).first;
        } else {
            // replay: advance the buffer roles exactly as the capture did
            *cur = c->graph_end_psi[key];
        }
        if (c->graph_end_psi.find(key) == c->graph_end_psi.end()) c->graph_end_psi[key] = *cur;
        hipError_t e = hipGraphLaunch(it->second, c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "hipGraphLaunch");
    }
    if (*cur != static_cast<void*>(c->d_state)) {
        hipError_t e = launch_copy(c->prec, c->geom(kReduceTiles), *cur, c->d_state, c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "final state copy");
        *cur = c->d_state;
    }
    return TDSE_OK;
}

// One Taylor step of order `order` (Horner form) on the psi held in `cur`.
// psi rotates through three buffers (the state and work vectors 0 and 1):
// launches alternate between the two buffers that do not hold psi, no launch
// writes a buffer it reads, and `cur` moves to the buffer that holds the new
// psi (run_steps copies it back into the state at the end).  With fuse_k = 0
// each Horner term is one sweep; with fuse_k = K each launch of the fused
// kernel (LDS-ring or wave-strip) does K terms (the last one the remainder).
hipError_t taylor_step_launches(tdse_ctx* c, const double* step, int order, void*& cur)
{
    const int S = c->stencil == 3 ? 1 : 2;
    void* free_bufs[2];
    int nf = 0;
    for (void* b : {static_cast<void*>(c->d_state), static_cast<void*>(c->d_vec(0)), static_cast<void*>(c->d_vec(1))})
        if (b != cur && nf < 2) free_bufs[nf++] = b;
    const void* psi = cur;
    const void* in = cur;
    void* out = nullptr;
    const int K = (c->gauge != 0) ? 0 : c->fuse_k;   // the fused kernels couple in the length gauge only
    if (K > 0) {
        const bool strips = c->fuse_kind >= 1;
        const bool pairs = c->fuse_kind >= 2;
        // strips take the tiles most rows first (a persistent launch from
        // the work queue, else one workgroup per tile in that order)
        unsigned* queue = (c->fuse_kind == 3) ? c->d_queue() : nullptr;
        const int32_t* perm = strips ? c->d_perm() : nullptr;
        SweepGeom gf = c->geom(strips ? kStripTiles : kFusedTiles);
        if (strips) gf.variant = K;   // the term count the strip tiles were built for
        int which = 0;
        for (int first = order; first >= 1; first -= K) {
            const int terms = std::min(K, first);
            out = free_bufs[which];
            // the step's last launch on strips also sums the main observables
            // when the step loop asks for them
            double* obs = (strips && first <= K) ? c->obs_req : nullptr;
            hipError_t e;
            {
                TimedLaunch tl(c, 5);
                e = pairs ? launch_horner_pstrip(c->prec, S, terms, gf, in, psi, out, step, first, c->stream, obs,
                                                 queue, perm)
                    : strips ? launch_horner_strip(c->prec, S, terms, gf, in, psi, out, step, first, c->stream, obs,
                                                   perm)
                             : launch_horner_fused(c->prec, S, terms, gf, in, psi, out, step, first, c->stream);
            }
            if (obs && e == hipSuccess) c->obs_main_done = true;
            if (e != hipSuccess) return e;
            in = out;
            which ^= 1;
        }
        cur = out;
        return hipSuccess;
    }
    // Horner: w = psi + (-i dt/P) H psi; w = psi + (-i dt/k) H w, k = P-1..1
    const SweepGeom g = c->hgeom();
    for (int k = order; k >= 1; --k) {
        out = free_bufs[(order - k) & 1];
        hipError_t e;
        {
            TimedLaunch tl(c, 0);
            e = launch_hsweep(c->prec, S, g, in, psi, out, step, k, c->stream);
        }
        if (e != hipSuccess) return e;
        in = out;
    }
    cur = out;
    return hipSuccess;
}

}  // namespace

// ---------------------------------------------------------------------------
// the hot path
// ---------------------------------------------------------------------------
extern "C" tdse_status tdse_apply_H(tdse_ctx* c, const double* e_field, const void* d_in, void* d_out)
{
    if (!c) return TDSE_E_INVALID;
    if (!c->bound) return c->fail(TDSE_E_UNBOUND, "tdse_apply_H: not bound");
    if (!e_field || !d_in || !d_out) return c->fail(TDSE_E_INVALID, "tdse_apply_H: null argument");
    const char* a = static_cast<const char*>(d_in);
    const char* b = static_cast<const char*>(d_out);
    const size_t nb = c->state_bytes();
    if (a < b + nb && b < a + nb) return c->fail(TDSE_E_INVALID, "tdse_apply_H: in and out overlap");
    std::vector<tdse_pulse> none(c->n_inst);
    std::vector<double> zero(c->n_inst, 0.0), one(c->n_inst, 1.0);
    // slot kEMid carries the caller's field values
    tdse_status st = upload_steps(c, nullptr, zero.data(), one.data(), 0, 1, 0);
    if (st != TDSE_OK) return st;
    hipError_t e = hipMemcpyAsync(c->d_step() + kEMid * c->n_inst, e_field, sizeof(double) * c->n_inst,
                                  hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "tdse_apply_H field upload");
    e = hipStreamSynchronize(c->stream);  // e_field is pageable caller memory
    if (e != hipSuccess) return c->hip_fail(e, "tdse_apply_H sync");
    TimedLaunch tl(c, 4);
    e = launch_hsweep(c->prec, c->stencil == 3 ? 1 : 2, c->hgeom(), d_in, nullptr, d_out, c->d_step(), 0,
                      c->stream);
    return (e == hipSuccess) ? TDSE_OK : c->hip_fail(e, "tdse_apply_H launch");
}

extern "C" tdse_status tdse_step_taylor(tdse_ctx* c, const tdse_pulse* pulses, const double* t0,
                                        const double* dt, int32_t order, int32_t nsteps,
                                        int32_t obs_every, tdse_obs* d_obs)
{
    if (!c) return TDSE_E_INVALID;
    if (order < 1 || order > 16) return c->fail(TDSE_E_INVALID, "tdse_step_taylor: order must be 1..16");
    tdse_status st = check_common(c, pulses, t0, dt, nsteps, obs_every, d_obs, TDSE_METHOD_TAYLOR, order);
    if (st != TDSE_OK) return st;
    st = check_stable(c, pulses, dt, order);
    if (st != TDSE_OK) return st;
    void* cur = c->d_state;
    const int64_t key = 1000 + 100 * c->fuse_k + 20 * c->fuse_kind + order;
    // the Taylor rotation never writes the buffer holding psi at the start of
    // a step, so the observables may overlap the next step
    return run_steps(c, pulses, t0, dt, nsteps, obs_every, d_obs, key, &cur,
                     [&](const double* step) { return taylor_step_launches(c, step, order, cur); }, true);
}

// Sec. 4 "Ground state calculation": field-free diffusion steps (imaginary
// time), each the order-P Taylor polynomial of exp(-dtau H) in Horner form (one
// launch per term, one radius per thread), then the norm of the result, the
// energy estimate -ln(n2)/(2 dtau) and the renormalisation into the state.
extern "C" tdse_status tdse_step_imag(tdse_ctx* c, const double* dtau, int32_t order, int32_t nsteps,
                                      double* d_energy)
{
    if (!c) return TDSE_E_INVALID;
    if (!c->bound) return c->fail(TDSE_E_UNBOUND, "tdse_step_imag: not bound");
    if (!dtau) return c->fail(TDSE_E_INVALID, "tdse_step_imag: null argument");
    if (order < 1 || order > 16) return c->fail(TDSE_E_INVALID, "tdse_step_imag: order must be 1..16");
    if (nsteps < 0) return c->fail(TDSE_E_INVALID, "tdse_step_imag: nsteps < 0");
    const size_t need = tdse_workspace_bytes(c, TDSE_METHOD_TAYLOR, order);
    if (c->work_bytes < need)
        return c->fail(TDSE_E_WORKSPACE, "tdse_step_imag: workspace too small (" + std::to_string(need) +
                                             " bytes needed)");
    const double xp = tdse_taylor_real_stability_limit(order);
    for (int k = 0; k < c->n_inst; ++k) {
        if (!(dtau[k] > 0.0) || !std::isfinite(dtau[k])) return c->fail(TDSE_E_INVALID, "tdse_step_imag: dtau must be > 0");
        const double lam = cached_bound(c, k, 0.0);
        if (dtau[k] * lam > xp) {
            char buf[256];
            std::snprintf(buf, sizeof buf,
                          "instance %d: dtau*lambda_max = %.4g exceeds the order-%d real-axis limit %.4g", k,
                          dtau[k] * lam, order, xp);
            return c->fail(TDSE_E_UNSTABLE, buf);
        }
    }
    c->drop_graphs();
    // one table of step scalars serves every step: no field, dt = dtau
    std::vector<double> zero(c->n_inst, 0.0);
    tdse_status st = upload_steps(c, nullptr, zero.data(), dtau, 0, 1, 0);
    if (st != TDSE_OK) return st;
    const int S = c->stencil == 3 ? 1 : 2;
    SweepGeom gs = c->geom(kSweepTiles);   // one radius per thread (variant 0)
    gs.gauge = 0;                          // no field: the gauge does not enter
    const SweepGeom red = c->geom(kReduceTiles);
    const double* step = c->d_step();
    double* part = c->d_partial();
    LanczosScalars* sc = c->d_lz();
    void* psi = c->d_state;
    void* v0 = c->d_vec(0);
    void* v1 = c->d_vec(1);
    // the input normalised first (no energy recorded)
    hipError_t e = launch_lz_norm(c->prec, red, psi, part, c->stream);
    if (e == hipSuccess) e = launch_imag_finish(red, part, step, 0, nullptr, 0, 0, sc, c->stream);
    if (e == hipSuccess) e = launch_imag_scale(c->prec, red, psi, v0, sc, c->stream);
    if (e == hipSuccess) e = launch_copy(c->prec, red, v0, psi, c->stream);
    for (int32_t s = 0; s < nsteps && e == hipSuccess; ++s) {
        // w_P = psi - dtau/P H psi, ..., w_1 = psi - dtau H w_2, alternating v0 / v1
        const void* in = psi;
        void* out = v0;
        for (int k = order; k >= 1 && e == hipSuccess; --k) {
            e = launch_hsweep(c->prec, S, gs, in, psi, out, step, -k, c->stream);
            in = out;
            out = (out == v0) ? v1 : v0;
        }
        if (e == hipSuccess) e = launch_lz_norm(c->prec, red, in, part, c->stream);
        if (e == hipSuccess) e = launch_imag_finish(red, part, step, 1, d_energy, nsteps, s, sc, c->stream);
        if (e == hipSuccess) e = launch_imag_scale(c->prec, red, in, psi, sc, c->stream);
    }
    return (e == hipSuccess) ? TDSE_OK : c->hip_fail(e, "tdse_step_imag");
}

extern "C" tdse_status tdse_step_rk4(tdse_ctx* c, const tdse_pulse* pulses, const double* t0,
                                     const double* dt, int32_t nsteps, int32_t obs_every,
                                     tdse_obs* d_obs)
{
    if (!c) return TDSE_E_INVALID;
    tdse_status st = check_common(c, pulses, t0, dt, nsteps, obs_every, d_obs, TDSE_METHOD_RK4, 4);
    if (st != TDSE_OK) return st;
    st = check_stable(c, pulses, dt, 4);
    if (st != TDSE_OK) return st;
    const int S = c->stencil == 3 ? 1 : 2;
    if (c->rk4_fused && c->gauge == 0) {
        // one strip launch per step; psi rotates through the state and work
        // vectors 0 and 1 (a launch writes a buffer it does not read, and the
        // buffer holding psi(s) is first overwritten in step s+2), so the
        // observables may overlap the next step
        SweepGeom g4 = c->geom(kRk4Tiles);
        g4.variant = 4;
        void* cur = c->d_state;
        return run_steps(c, pulses, t0, dt, nsteps, obs_every, d_obs, 2001, &cur, [&](const double* step) {
            void* out = nullptr;
            for (void* b : {static_cast<void*>(c->d_state), static_cast<void*>(c->d_vec(0)),
                            static_cast<void*>(c->d_vec(1))})
                if (b != cur && !out) out = b;
            hipError_t e;
            {
                TimedLaunch tl(c, 6);
                e = launch_rk4_strip(c->prec, S, g4, cur, out, step, c->stream);
            }
            if (e == hipSuccess) cur = out;
            return e;
        }, true);
    }
    const SweepGeom g = c->geom();
    void* psi = c->d_state;
    void* ga = c->d_vec(0);
    void* gb = c->d_vec(1);
    void* acc = c->d_vec(2);
    void* cur = psi;
    return run_steps(c, pulses, t0, dt, nsteps, obs_every, d_obs, 2000, &cur, [&](const double* step) {
        const void* gin[4] = {psi, ga, gb, ga};
        void* gout[4] = {ga, gb, ga, nullptr};
        for (int s = 0; s < 4; ++s) {
            TimedLaunch tl(c, 1);
            hipError_t e = launch_rk4_stage(c->prec, S, g, s, gin[s], psi, acc, gout[s], step, c->stream);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    });
}

extern "C" double tdse_rk_stability_limit(int32_t method)
{
    const RkTableau* T = rk_tableau(method);
    if (!T) return 0.0;
    // R(z) = 1 + sum_k gamma_k z^k, gamma_k = b^T A^(k-1) 1: the step's factor
    // on dy/dt = lambda y; the largest y with |R(i y')| <= 1 + 1e-12 up to y
    double gamma[kRkMax + 1] = {1.0};
    double v[kRkMax];
    for (int i = 0; i < T->stages; ++i) v[i] = 1.0;
    for (int k = 1; k <= T->stages; ++k) {
        double g = 0.0;
        for (int i = 0; i < T->stages; ++i) g += T->b[i] * v[i];
        gamma[k] = g;
        double w[kRkMax];
        for (int i = 0; i < T->stages; ++i) {
            w[i] = 0.0;
            for (int j = 0; j < T->stages; ++j) w[i] += T->a[i][j] * v[j];
        }
        for (int i = 0; i < T->stages; ++i) v[i] = w[i];
    }
    auto mag = [&](double y) {
        std::complex<double> z(0.0, y), zk(1.0, 0.0), r(1.0, 0.0);
        for (int k = 1; k <= T->stages; ++k) {
            zk *= z;
            r += gamma[k] * zk;
        }
        return std::abs(r);
    };
    const double tol = 1.0 + 1e-12;
    double y = 0.0;
    const double h = 1e-4;
    while (y < 10.0 && mag(y + h) <= tol) y += h;
    double a = y, b = y + h;
    for (int i = 0; i < 60; ++i) {
        const double mid = 0.5 * (a + b);
        if (mag(mid) <= tol) a = mid; else b = mid;
    }
    return a;
}

// Appendix "Runge-Kutta" (eq. RKDeriv): one launch per stage over the sweep
// tiles; psi rotates through the state and work vectors 0 and 1 as in the
// Taylor path (stage 0 reads psi, stage i reads g_i from one of the two other
// buffers and writes g_{i+1} to the other; the last stage writes the new psi
// there), the stage derivatives k_0..k_{S-2} sit in work vectors 2..S.
extern "C" tdse_status tdse_step_rk(tdse_ctx* c, const tdse_pulse* pulses, const double* t0, const double* dt,
                                    int32_t method, int32_t nsteps, int32_t obs_every, tdse_obs* d_obs,
                                    double* d_sigma)
{
    if (!c) return TDSE_E_INVALID;
    const RkTableau* T = rk_tableau(method);
    if (!T) return c->fail(TDSE_E_INVALID, "tdse_step_rk: unknown method");
    tdse_status st = check_common(c, pulses, t0, dt, nsteps, obs_every, d_obs, TDSE_METHOD_RK_TABLEAU, method);
    if (st != TDSE_OK) return st;
    const double y = tdse_rk_stability_limit(method);
    for (int k = 0; k < c->n_inst; ++k) {
        const double lam = cached_bound(c, k, coupling_bound(c, pulses[k]));
        if (dt[k] * lam > y) {
            char buf[256];
            std::snprintf(buf, sizeof buf,
                          "instance %d: dt*lambda_max = %.4g exceeds the method's stability limit %.4g", k,
                          dt[k] * lam, y);
            return c->fail(TDSE_E_UNSTABLE, buf);
        }
    }
    bool pair = false;
    for (int i = 0; i < T->stages; ++i) pair = pair || T->bhat[i] != 0.0;
    const bool err = pair && d_sigma != nullptr;
    // the stage times the step table carries (captured graphs depend on them
    // only through the uploaded values)
    c->rk_stages = T->stages;
    for (int i = 0; i < kRkMax; ++i) c->rk_c[i] = (i < T->stages) ? T->c[i] : 0.0;
    const int S = c->stencil == 3 ? 1 : 2;
    const SweepGeom g = c->geom();
    void* kv = c->d_vec(2);
    const int nk = T->stages - 1;
    // k vectors: one state-shaped vector apart (48-bit: plane by plane)
    const int64_t kstride = (c->prec == TDSE_FP48) ? c->plane() : (int64_t)(c->state_bytes() / c->elem);
    double* part = c->d_partial();
    void* cur = c->d_state;
    const int64_t key = 4000 + 10 * method + (err ? 1 : 0) + (int64_t)reinterpret_cast<uintptr_t>(d_sigma) * 100;
    st = run_steps(c, pulses, t0, dt, nsteps, obs_every, d_obs, key, &cur, [&](const double* step) {
        void* bufs[2];
        int nb = 0;
        for (void* b : {static_cast<void*>(c->d_state), static_cast<void*>(c->d_vec(0)), static_cast<void*>(c->d_vec(1))})
            if (b != cur && nb < 2) bufs[nb++] = b;
        const void* gin = cur;
        void* out = nullptr;
        for (int i = 0; i < T->stages; ++i) {
            RkStage a{};
            a.stage = i;
            a.last = (i == T->stages - 1) ? 1 : 0;
            a.err = (a.last && err) ? 1 : 0;
            a.slot = kEStage0 + i;
            for (int j = 0; j <= i; ++j) {
                // g_{i+1} = psi + dt sum_j a_{i+1,j} k_j, or the new state
                a.w[j] = a.last ? T->b[j] : T->a[i + 1][j];
                a.we[j] = T->b[j] - T->bhat[j];
            }
            out = bufs[i & 1];
            hipError_t e;
            {
                TimedLaunch tl(c, 1);
                e = launch_rk_stage(c->prec, S, g, gin, cur, kv, kstride, nk, out, step, a, part, c->stream);
            }
            if (e != hipSuccess) return e;
            gin = out;
        }
        if (err) {
            hipError_t e = launch_rk_sigma(g, part, d_sigma, c->stream);
            if (e != hipSuccess) return e;
        }
        cur = out;
        return hipSuccess;
    });
    c->rk_stages = 0;
    return st;
}

extern "C" tdse_status tdse_step_lanczos(tdse_ctx* c, const tdse_pulse* pulses, const double* t0,
                                         const double* dt, int32_t m, int32_t nsteps,
                                         int32_t obs_every, tdse_obs* d_obs)
{
    if (!c) return TDSE_E_INVALID;
    if (m < 1 || m > kMaxKrylov) return c->fail(TDSE_E_INVALID, "tdse_step_lanczos: m must be 1..64");
    tdse_status st = check_common(c, pulses, t0, dt, nsteps, obs_every, d_obs, TDSE_METHOD_LANCZOS, m);
    if (st != TDSE_OK) return st;
    const int S = c->stencil == 3 ? 1 : 2;
    const SweepGeom g = c->geom(kReduceTiles);
    void* psi = c->d_state;
    void* w = c->d_vec(0);
    void* basis = c->d_vec(1);  // vectors 1..m-1
    // element distance of consecutive basis vectors (48-bit storage: the
    // basis vectors are stored plane by plane, one plane length apart)
    const int64_t stride = (c->prec == TDSE_FP48) ? c->plane() : (int64_t)(c->state_bytes() / c->elem);
    LanczosScalars* sc = c->d_lz();
    double* part = c->d_partial();
    void* cur = psi;
    // the breakdown report of this call starts from the requested dimension
    hipError_t er = launch_lz_reset(g, m, sc, c->stream);
    if (er != hipSuccess) return c->hip_fail(er, "tdse_step_lanczos reset");
    c->lz_m = m;
    return run_steps(c, pulses, t0, dt, nsteps, obs_every, d_obs, 3000 + m, &cur, [&](const double* step) {
        hipError_t e = launch_lz_norm(c->prec, g, psi, part, c->stream);
        if (e == hipSuccess) e = launch_lz_norm_finish(g, part, sc, c->stream);
        for (int j = 0; j < m && e == hipSuccess; ++j) {
            {
                TimedLaunch tl(c, 3);
                e = launch_lz_sweep_a(c->prec, S, g, j, m, psi, basis, stride, w, step, sc, part, c->stream);
            }
            if (e == hipSuccess) e = launch_lz_finish_a(g, j, m, part, sc, c->stream);
            if (j + 1 < m) {
                if (e == hipSuccess) e = launch_lz_sweep_b(c->prec, g, j, m, psi, basis, stride, w, sc, part, c->stream);
                if (e == hipSuccess) e = launch_lz_finish_b(g, j, part, sc, c->stream);
            }
        }
        if (e == hipSuccess) e = launch_lz_expm(g, step, sc, c->stream);
        if (e == hipSuccess) e = launch_lz_recombine(c->prec, g, m, psi, basis, stride, sc, c->stream);
        return e;
    });
}

extern "C" tdse_status tdse_observables(tdse_ctx* c, const tdse_pulse* pulses, const double* t,
                                        tdse_obs* host_out)
{
    if (!c) return TDSE_E_INVALID;
    if (!c->bound) return c->fail(TDSE_E_UNBOUND, "tdse_observables: not bound");
    if (!pulses || !t || !host_out) return c->fail(TDSE_E_INVALID, "tdse_observables: null argument");
    // one pseudo-step whose end is t: t0 = t - dt with dt = 1 gives t_end = t
    std::vector<double> t0(c->n_inst), one(c->n_inst, 1.0);
    for (int k = 0; k < c->n_inst; ++k) t0[k] = t[k] - 1.0;
    tdse_status st = upload_steps(c, pulses, t0.data(), one.data(), 0, 1, 1);
    if (st != TDSE_OK) return st;
    // the exact time t (not (t - 1) + 1) goes into the record
    double* tmp = reinterpret_cast<double*>(c->d_work + c->off_obs_tmp);
    hipError_t e = hipMemcpyAsync(c->d_step() + kTEnd * c->n_inst, t, sizeof(double) * c->n_inst,
                                  hipMemcpyHostToDevice, c->stream);
    std::vector<double> ee(c->n_inst);
    for (int k = 0; k < c->n_inst; ++k) ee[k] = field_at(pulses[k], t[k]);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_step() + kEObs * c->n_inst, ee.data(), sizeof(double) * c->n_inst,
                           hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_obs(c, c->d_state, c->d_step(), tmp, kObsRecord, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host_out, tmp, sizeof(tdse_obs) * c->n_inst, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "tdse_observables");
    for (int k = 0; k < c->n_inst; ++k)
        if (!std::isfinite(host_out[k].norm)) return c->fail(TDSE_E_NONFINITE, "tdse_observables: norm is not finite");
    return TDSE_OK;
}

// ---------------------------------------------------------------------------
// observables without a workspace for scratch: a static device buffer
// ---------------------------------------------------------------------------
// The scratch of tdse_observables_noalloc: the call's step scalars, the
// per-tile partial sums and the records before their copy to the host.  One
// copy per GPU (the runtime loads the code object on each device used), held
// until the process ends.  Host code never passes the array's name to a
// kernel or a copy: it takes the device address from hipGetSymbolAddress, per
// device (scratch_ptr).
static __device__ __align__(256) char scratch[TDSE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with the device current).
hipError_t scratch_ptr(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Byte layout of the scratch for a context: [step scalars | partial sums |
// records], each region 256-byte aligned.
struct NoallocLayout {
    size_t step = 0, partial = 0, records = 0, total = 0;
};
NoallocLayout noalloc_layout(const tdse_ctx* c)
{
    NoallocLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, kAlign);
        return at;
    };
    L.step = take(sizeof(double) * kSlots * (size_t)c->n_inst);
    L.partial = take(sizeof(double) * ((size_t)c->tiles[kObsTiles].size() * kObsMainQ +
                                       (size_t)c->tiles[kPopTiles].size() * kObsPopQ));
    L.records = take(sizeof(tdse_obs) * (size_t)c->n_inst);
    L.total = o;
    return L;
}
}  // namespace

extern "C" tdse_status tdse_observables_noalloc(tdse_ctx* c, const tdse_pulse* pulses, const double* t,
                                                tdse_obs* host_out)
{
    if (!c) return TDSE_E_INVALID;
    const NoallocLayout L = noalloc_layout(c);
    if (L.total > (size_t)TDSE_NOALLOC_SCRATCH_BYTES)
        return c->fail(TDSE_E_WORKSPACE, "tdse_observables_noalloc: the grids need " + std::to_string(L.total) +
                                             " bytes of scratch, more than the static " +
                                             std::to_string((size_t)TDSE_NOALLOC_SCRATCH_BYTES));
    if (!c->bound) return c->fail(TDSE_E_UNBOUND, "tdse_observables_noalloc: not bound");
    if (!pulses || !t || !host_out) return c->fail(TDSE_E_INVALID, "tdse_observables_noalloc: null argument");
    void* base = nullptr;
    hipError_t e = scratch_ptr(&base);
    if (e != hipSuccess) return c->hip_fail(e, "tdse_observables_noalloc: scratch address");
    char* sb = static_cast<char*>(base);
    double* d_step = reinterpret_cast<double*>(sb + L.step);
    double* d_partial = reinterpret_cast<double*>(sb + L.partial);
    double* d_rec = reinterpret_cast<double*>(sb + L.records);
    // the step scalars of one record at time t (the fields the finish reads:
    // t, E(t), record index 0), staged in the context's pinned buffer; every
    // scratch value a kernel reads is written first in this call, so nothing
    // needs clearing
    const int b = c->step_buf;
    c->step_buf ^= 1;
    if (c->step_ev_used[b]) {
        e = hipEventSynchronize(c->step_ev[b]);
        if (e != hipSuccess) return c->hip_fail(e, "tdse_observables_noalloc: staging wait");
    }
    double* h = c->h_step[b];
    const int n = c->n_inst;
    for (int k = 0; k < n; ++k) {
        h[kEStart * n + k] = 0.0;
        h[kEMid * n + k] = 0.0;
        h[kEEnd * n + k] = 0.0;
        h[kEObs * n + k] = field_at(pulses[k], t[k]);
        h[kTEnd * n + k] = t[k];
        h[kDt * n + k] = 1.0;
        h[kRec * n + k] = 0.0;
    }
    e = hipMemcpyAsync(d_step, h, sizeof(double) * kSlots * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->step_ev[b], c->stream);
    if (e == hipSuccess) c->step_ev_used[b] = true;
    if (e == hipSuccess) e = launch_obs(c, c->d_state, d_step, d_rec, kObsRecord, c->stream, d_partial);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host_out, d_rec, sizeof(tdse_obs) * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "tdse_observables_noalloc");
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(host_out[k].norm))
            return c->fail(TDSE_E_NONFINITE, "tdse_observables_noalloc: norm is not finite");
    return TDSE_OK;
}

extern "C" tdse_status tdse_set_gauge(tdse_ctx* c, int32_t gauge)
{
    if (!c) return TDSE_E_INVALID;
    if (gauge != TDSE_GAUGE_LENGTH && gauge != TDSE_GAUGE_VELOCITY)
        return c->fail(TDSE_E_INVALID, "tdse_set_gauge: gauge must be TDSE_GAUGE_LENGTH or TDSE_GAUGE_VELOCITY");
    if (gauge != c->gauge) c->drop_graphs();
    c->gauge = gauge;
    return TDSE_OK;
}

extern "C" int32_t tdse_gauge(const tdse_ctx* c) { return c ? c->gauge : 0; }

static tdse_status upload_inst(tdse_ctx* c, const char* what)
{
    c->drop_graphs();
    hipError_t e = hipMemcpyAsync(c->d_work + c->off_inst, c->inst.data(), sizeof(Inst) * c->inst.size(),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return (e == hipSuccess) ? TDSE_OK : c->hip_fail(e, what);
}

extern "C" tdse_status tdse_set_absorber(tdse_ctx* c, const double* r_abs, const double* p_abs)
{
    if (!c) return TDSE_E_INVALID;
    if (!c->bound) return c->fail(TDSE_E_UNBOUND, "tdse_set_absorber: not bound");
    if (!r_abs || !p_abs) return c->fail(TDSE_E_INVALID, "tdse_set_absorber: null argument");
    for (int k = 0; k < c->n_inst; ++k)
        if (!std::isfinite(r_abs[k]) || (r_abs[k] > 0.0 && !(p_abs[k] > 0.0 && std::isfinite(p_abs[k]))))
            return c->fail(TDSE_E_INVALID, "tdse_set_absorber: instance " + std::to_string(k) +
                                               ": r_abs must be finite, p_abs finite and > 0 where r_abs > 0");
    bool on = false;
    for (int k = 0; k < c->n_inst; ++k) {
        const bool a = r_abs[k] > 0.0;
        c->inst[k].r_abs = a ? r_abs[k] : 0.0;
        c->inst[k].p_abs = a ? p_abs[k] : 0.0;
        on = on || a;
    }
    c->absorber_on = on;
    return upload_inst(c, "tdse_set_absorber");
}

extern "C" tdse_status tdse_set_flux(tdse_ctx* c, const int32_t* i_flux)
{
    if (!c) return TDSE_E_INVALID;
    if (!c->bound) return c->fail(TDSE_E_UNBOUND, "tdse_set_flux: not bound");
    if (!i_flux) return c->fail(TDSE_E_INVALID, "tdse_set_flux: null argument");
    for (int k = 0; k < c->n_inst; ++k)
        if (i_flux[k] < -1 || i_flux[k] >= c->inst[k].n)
            return c->fail(TDSE_E_INVALID, "tdse_set_flux: instance " + std::to_string(k) +
                                               ": i_flux must be -1 or a radial index of the grid");
    bool on = false;
    for (int k = 0; k < c->n_inst; ++k) {
        c->inst[k].i_flux = i_flux[k];
        on = on || i_flux[k] >= 0;
    }
    c->flux_on = on;
    hipError_t e = hipMemsetAsync(c->d_jprev(), 0, sizeof(double) * 2 * (size_t)c->n_inst, c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "tdse_set_flux");
    return upload_inst(c, "tdse_set_flux");
}

extern "C" tdse_status tdse_get_flux(tdse_ctx* c, double* host_yield)
{
    if (!c) return TDSE_E_INVALID;
    if (!c->bound) return c->fail(TDSE_E_UNBOUND, "tdse_get_flux: not bound");
    if (!host_yield) return c->fail(TDSE_E_INVALID, "tdse_get_flux: null argument");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = hipMemcpy(host_yield, c->d_yield(), sizeof(double) * (size_t)c->n_inst, hipMemcpyDeviceToHost);
    return (e == hipSuccess) ? TDSE_OK : c->hip_fail(e, "tdse_get_flux");
}

extern "C" tdse_status tdse_lanczos_dims(tdse_ctx* c, int32_t* host_meff)
{
    if (!c || !host_meff) return TDSE_E_INVALID;
    if (!c->bound) return c->fail(TDSE_E_UNBOUND, "tdse_lanczos_dims: not bound");
    if (c->lz_m <= 0) return c->fail(TDSE_E_INVALID, "tdse_lanczos_dims: no Lanczos step since the context was bound");
    std::vector<LanczosScalars> sc(c->n_inst);
    hipError_t e = hipMemcpyAsync(sc.data(), c->d_lz(), sizeof(LanczosScalars) * c->n_inst, hipMemcpyDeviceToHost,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "tdse_lanczos_dims");
    bool broke = false;
    for (int k = 0; k < c->n_inst; ++k) {
        host_meff[k] = sc[k].meff_min;
        broke = broke || sc[k].meff_min < c->lz_m;
    }
    if (broke) return c->fail(TDSE_E_BREAKDOWN, "tdse_lanczos_dims: the Krylov process stopped early (invariant subspace)");
    return TDSE_OK;
}

// A rebuilt tile set and the instance table (it holds each instance's tile
// range of every set: the observables' finish reads the ranges).
static hipError_t upload_tiles(tdse_ctx* c, int set)
{
    if (c->tiles[set].size() > c->tile_cap[set]) return hipErrorInvalidValue;   // never past the region
    hipError_t e = hipMemcpyAsync(c->d_work + c->off_tiles[set], c->tiles[set].data(),
                                  sizeof(Tile) * c->tiles[set].size(), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && set == kStripTiles && !c->strip_perm.empty())
        e = hipMemcpyAsync(c->d_perm(), c->strip_perm.data(), sizeof(int32_t) * c->strip_perm.size(),
                           hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_work + c->off_inst, c->inst.data(), sizeof(Inst) * c->inst.size(),
                           hipMemcpyHostToDevice, c->stream);
    return e;
}

// The autotuners time the length-gauge kernels (the velocity gauge runs the
// workgroup sweeps in a fixed shape): the context is in the length gauge
// while they run.
struct LengthGaugeScope {
    tdse_ctx* c;
    int saved;
    explicit LengthGaugeScope(tdse_ctx* ctx) : c(ctx), saved(ctx->gauge) { c->gauge = 0; }
    ~LengthGaugeScope()
    {
        if (saved != 0) c->drop_graphs();
        c->gauge = saved;
    }
};

extern "C" tdse_status tdse_autotune(tdse_ctx* c, int32_t* rows_out)
{
    if (!c) return TDSE_E_INVALID;
    LengthGaugeScope lgs(c);
    if (!c->bound) return c->fail(TDSE_E_UNBOUND, "tdse_autotune: not bound");
    if (c->work_bytes < tdse_workspace_bytes(c, TDSE_METHOD_TAYLOR, 2))
        return c->fail(TDSE_E_WORKSPACE, "tdse_autotune: needs the Taylor workspace (two vectors)");
    std::vector<double> zero(c->n_inst, 0.0), one(c->n_inst, 1.0);
    tdse_status st = upload_steps(c, nullptr, zero.data(), one.data(), 0, 1, 0);
    if (st != TDSE_OK) return st;
    const int S = c->stencil == 3 ? 1 : 2;
    void* psi = c->d_state;
    void* out = c->d_vec(0);
    void* ref = c->d_vec(1);
    unsigned int* counter = reinterpret_cast<unsigned int*>(c->d_work + c->off_obs_tmp);
    const int start_rows = c->rows_sweep;
    const int start_variant = c->sweep_variant;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // reference sweep with the current tiles
    if (e == hipSuccess) e = launch_hsweep(c->prec, S, c->hgeom(), psi, psi, ref, c->d_step(), 1, c->stream);
    double best_ms = 1e300;
    int best = start_rows, best_variant = start_variant;
    const int cands[] = {1, 2, 4, 8, 16, 32};
    // rows x variant (bit 0: two radii per thread, bit 1: XCD-contiguous
    // order, bit 2: wave strips of one level; with bit 2, bit 0 is unused)
    const int variants[] = {0, 1, 2, 3, 4, 6};
    for (int cand = 0; cand < 36; ++cand) {
        const int rows = cands[cand % 6];
        const int variant = variants[cand / 6];
        if (e != hipSuccess) break;
        if (rows != 1 && c->total_cols / rows < 64) continue;
        if (c->prec == TDSE_FP48 && (variant & 5) == 1) continue;   // two-radii sweeps: FP64/FP32 storage only
        c->sweep_variant = variant;
        const int set = (variant & 4) ? kApplyTiles : (variant & 1) ? kPairTiles : kSweepTiles;
        build_tiles(c, set, rows);
        e = upload_tiles(c, set);
        const SweepGeom g = c->hgeom();
        for (int w = 0; w < 2 && e == hipSuccess; ++w)
            e = launch_hsweep(c->prec, S, g, psi, psi, out, c->d_step(), 1, c->stream);
        const int reps = 20;
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r)
            e = launch_hsweep(c->prec, S, g, psi, psi, out, c->d_step(), 1, c->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(counter, 0, sizeof(unsigned int), c->stream);
        if (e == hipSuccess) e = launch_count_diff(c->prec, c->geom(kReduceTiles), out, ref, counter, c->stream);
        unsigned int diff = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&diff, counter, sizeof diff, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) break;
        if (diff != 0) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            build_tiles(c, kSweepTiles, start_rows);
            build_tiles(c, kPairTiles, start_rows);
            build_tiles(c, kApplyTiles, start_rows);
            c->sweep_variant = start_variant;
            (void)upload_tiles(c, kSweepTiles);
            (void)upload_tiles(c, kPairTiles);
            (void)upload_tiles(c, kApplyTiles);
            (void)hipStreamSynchronize(c->stream);
            return c->fail(TDSE_E_HIP, "tdse_autotune: a tile shape changed the result of a sweep (" +
                                           std::to_string(diff) + " elements, rows " + std::to_string(rows) +
                                           ", variant " + std::to_string(variant) + ")");
        }
        if (ms / reps < best_ms) {
            best_ms = ms / reps;
            best = rows;
            best_variant = variant;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    build_tiles(c, kSweepTiles, (e == hipSuccess) ? best : start_rows);
    build_tiles(c, kPairTiles, (e == hipSuccess) ? best : start_rows);
    build_tiles(c, kApplyTiles, (e == hipSuccess) ? best : start_rows);
    c->sweep_variant = (e == hipSuccess) ? best_variant : start_variant;
    hipError_t e2 = upload_tiles(c, kSweepTiles);
    if (e2 == hipSuccess) e2 = upload_tiles(c, kPairTiles);
    if (e2 == hipSuccess) e2 = upload_tiles(c, kApplyTiles);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return c->hip_fail(e, "tdse_autotune");
    if (e2 != hipSuccess) return c->hip_fail(e2, "tdse_autotune upload");
    c->rows_sweep = best;
    c->drop_graphs();
    tune_cache_store(c, best, best_variant);
    if (rows_out) *rows_out = best;
    return TDSE_OK;
}

extern "C" tdse_status tdse_autotune_taylor(tdse_ctx* c, int32_t order, int32_t* k_out, int32_t* rows_out)
{
    if (!c) return TDSE_E_INVALID;
    LengthGaugeScope lgs(c);
    if (!c->bound) return c->fail(TDSE_E_UNBOUND, "tdse_autotune_taylor: not bound");
    if (order < 1 || order > 16) return c->fail(TDSE_E_INVALID, "tdse_autotune_taylor: order must be 1..16");
    if (c->work_bytes < tdse_workspace_bytes(c, TDSE_METHOD_TUNE, 0))
        return c->fail(TDSE_E_WORKSPACE, "tdse_autotune_taylor: needs the TDSE_METHOD_TUNE workspace");
    // one step of stable dt with a field, for every instance
    const double y = tdse_taylor_stability_limit(order);
    std::vector<tdse_pulse> pulses(c->n_inst);
    std::vector<double> t0(c->n_inst, 0.0), dt(c->n_inst);
    for (int k = 0; k < c->n_inst; ++k) {
        pulses[k] = tdse_pulse{0.05, 1.0, 1.0, 0.0, -1.0};
        dt[k] = 0.5 * y / cached_bound(c, k, 0.05);
    }
    tdse_status st = upload_steps(c, pulses.data(), t0.data(), dt.data(), 0, 1, 0);
    if (st != TDSE_OK) return st;
    const SweepGeom red = c->geom(kReduceTiles);
    void* psi = c->d_state;
    void* backup = c->d_vec(2);
    void* ref = c->d_vec(3);
    double* acc = reinterpret_cast<double*>(c->d_work + c->off_obs_tmp);
    const int keep_k = c->fuse_k, keep_rows = c->rows_fused, keep_kind = c->fuse_kind;
    const bool keep_timing = c->timing;
    c->timing = false;
    hipError_t e = launch_copy(c->prec, red, psi, backup, c->stream);

    // reference: one launch per term
    auto one_step = [&](void** cur) -> hipError_t {
        *cur = psi;
        hipError_t ee = launch_copy(c->prec, red, backup, psi, c->stream);
        void* cc = psi;
        if (ee == hipSuccess) ee = taylor_step_launches(c, c->d_step(), order, cc);
        *cur = cc;
        return ee;
    };
    c->fuse_k = 0;
    void* cur = psi;
    if (e == hipSuccess) e = one_step(&cur);
    if (e == hipSuccess) e = launch_copy(c->prec, red, cur, ref, c->stream);

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // kind 0: LDS-ring kernel, kind 1: wave-strip kernel, kind 2: pair strips,
    // kind 3: pair strips in a persistent launch
    struct Cand { int k, rows, kind; };
    std::vector<Cand> cands = {{0, 0, 0}};
    for (int K = 2; K <= std::min(order, (int)kMaxFused); ++K) {
        if (c->prec != TDSE_FP48)   // the LDS-ring kernel has no 48-bit form
            for (int rows : {8, 16, 32}) cands.push_back({K, rows, 0});
        for (int rows : {8, 16, 32, 64}) cands.push_back({K, rows, 1});
        for (int rows : {8, 16, 32, 64}) cands.push_back({K, rows, 2});
        for (int rows : {16, 32, 64}) cands.push_back({K, rows, 3});
    }
    double best_ms = 1e300;
    Cand best = {0, keep_rows, keep_kind};
    std::string bad;
    std::set<std::pair<int, int>> failed;   // (K, kind) with a candidate that missed the reference
    std::map<int, std::pair<double, Cand>> best_strip;   // per K: the fastest strip candidate (ms, shape)
    for (const Cand& cd : cands) {
        if (e != hipSuccess) break;
        c->fuse_k = cd.k;
        c->fuse_kind = cd.kind;
        if (cd.k > 0) {
            const int set = cd.kind ? kStripTiles : kFusedTiles;
            c->rows_fused = cd.rows;
            build_tiles(c, set, cd.rows);
            e = upload_tiles(c, set);
        }
        // correctness against the reference step
        if (e == hipSuccess) e = one_step(&cur);
        if (e == hipSuccess) e = hipMemsetAsync(acc, 0, 2 * sizeof(double), c->stream);
        if (e == hipSuccess) e = launch_diff_norm(c->prec, red, cur, ref, acc, c->stream);
        double h_acc[2] = {0.0, 0.0};
        if (e == hipSuccess) e = hipMemcpyAsync(h_acc, acc, sizeof h_acc, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) break;
        const double rel = std::sqrt(h_acc[0] / std::max(h_acc[1], 1e-300));
        // FP64: bit for bit; otherwise the per-term step rounds every
        // intermediate level to the storage precision, the fused launches
        // only their outputs
        const double tol = (c->prec == TDSE_FP64) ? 0.0 : (c->prec == TDSE_FP48) ? 1e-9 : 1e-6;
        if (!(rel <= tol)) {
            bad += " K=" + std::to_string(cd.k) + "/rows=" + std::to_string(cd.rows) + "/kind=" +
                   std::to_string(cd.kind) + ": " + std::to_string(rel);
            failed.insert({cd.k, cd.kind});
            continue;
        }
        // timing: reps steps from the backed-up state
        const int reps = 10;
        e = launch_copy(c->prec, red, backup, psi, c->stream);
        cur = psi;
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = taylor_step_launches(c, c->d_step(), order, cur);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) break;
        if (ms / reps < best_ms) {
            best_ms = ms / reps;
            best = cd;
        }
        if (cd.kind >= 1) {
            auto it = best_strip.find(cd.k);
            if (it == best_strip.end() || ms / reps < it->second.first) best_strip[cd.k] = {ms / reps, cd};
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    // restore the state and the chosen configuration
    hipError_t e2 = launch_copy(c->prec, red, backup, psi, c->stream);
    c->fuse_k = (e == hipSuccess) ? best.k : keep_k;
    c->fuse_kind = (e == hipSuccess) ? best.kind : keep_kind;
    c->rows_fused = (e == hipSuccess && best.k > 0) ? best.rows : keep_rows;
    build_tiles(c, kFusedTiles, c->rows_fused);
    build_tiles(c, kStripTiles, c->rows_fused);
    if (e2 == hipSuccess) e2 = upload_tiles(c, kFusedTiles);
    if (e2 == hipSuccess) e2 = upload_tiles(c, kStripTiles);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->stream);
    // the observables, with the strip kernel chosen: time steps that record
    // after every step, the main sums in the step's last launch or in their
    // own pass (beside the next step, as the step loop runs them), and keep
    // the faster.  The records go to work vector 3 (free by now), when it
    // holds them.
    const int obs_reps = 8;
    if (e == hipSuccess && e2 == hipSuccess && c->fuse_k > 0 && c->fuse_kind >= 1 &&
        sizeof(double) * kObsRecord * obs_reps * (size_t)c->n_inst <= c->state_bytes()) {
        tdse_obs* rec = reinterpret_cast<tdse_obs*>(ref);
        const int64_t rec_stride = (int64_t)obs_reps * kObsRecord;
        const bool side = c->obs_overlap;
        if (side) e2 = ensure_obs_stream(c);
        hipEvent_t o0 = nullptr, o1 = nullptr;
        if (e2 == hipSuccess) e2 = hipEventCreate(&o0);
        if (e2 == hipSuccess) e2 = hipEventCreate(&o1);
        if (e2 == hipSuccess) {
            tdse_status su = upload_steps(c, pulses.data(), t0.data(), dt.data(), 0, obs_reps, 1);
            if (su != TDSE_OK) e2 = hipErrorUnknown;
        }
        // the strip heights the step timing tried, with both modes, and both
        // strip kernels: the launch with the sums does one more iteration
        // per tile, and the sums cost the two kernels differently, which can
        // move the best height and kernel
        const int chosen_rows = c->rows_fused, chosen_kind = c->fuse_kind, chosen_k = c->fuse_k;
        int best_rows = chosen_rows, best_kind = chosen_kind, best_k = chosen_k;
        bool best_fused = true;
        float best_obs_ms = 3.0e38f;
        std::vector<int> heights = {chosen_rows};
        for (int r : {16, 32, 64})
            if (r != chosen_rows) heights.push_back(r);
        struct Shape { int k, kind, rows; };
        std::vector<Shape> shapes;
        for (int kind : {chosen_kind, 1, 2, 3})
            if (kind == chosen_kind || failed.count({chosen_k, kind}) == 0) {
                bool seen = false;
                for (const Shape& sh : shapes) seen = seen || sh.kind == kind;
                if (!seen)
                    for (int rows : heights) shapes.push_back({chosen_k, kind, rows});
            }
        // the best strip shape of the two next-fastest term counts (the
        // observables in the last launch can reorder close term counts)
        std::vector<std::pair<double, Cand>> others;
        for (const auto& kv : best_strip)
            if (kv.first != chosen_k && failed.count({kv.first, kv.second.second.kind}) == 0)
                others.push_back(kv.second);
        std::sort(others.begin(), others.end(),
                  [](const std::pair<double, Cand>& a, const std::pair<double, Cand>& b) { return a.first < b.first; });
        for (size_t i = 0; i < others.size() && i < 2; ++i)
            shapes.push_back({others[i].second.k, others[i].second.kind, others[i].second.rows});
        for (const Shape& sh : shapes) {
            if (e2 != hipSuccess) break;
            const int rows = sh.rows;
            c->fuse_k = sh.k;
            c->fuse_kind = sh.kind;
            c->rows_fused = rows;
            build_tiles(c, kStripTiles, rows);
            e2 = upload_tiles(c, kStripTiles);
            // the fastest of 4 timed passes (pass 0 warms both up): the
            // minimum is steadier than a sum against other work on the box
            float ms_mode[2] = {3.0e38f, 3.0e38f};
            for (int pass = 0; pass < 5 && e2 == hipSuccess; ++pass) {
                for (int fused = 0; fused < 2 && e2 == hipSuccess; ++fused) {
                    c->obs_fusion = fused != 0;
                    void* oc = psi;
                    e2 = launch_copy(c->prec, red, backup, psi, c->stream);
                    auto fn = [&](const double* step) { return taylor_step_launches(c, step, order, oc); };
                    if (e2 == hipSuccess) e2 = hipEventRecord(o0, c->stream);
                    if (e2 == hipSuccess) e2 = enqueue_chunk(c, 0, obs_reps, 1, rec, rec_stride, &oc, fn, side, false);
                    if (e2 == hipSuccess) e2 = hipEventRecord(o1, c->stream);
                    if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->stream);
                    float ms = 0.0f;
                    if (e2 == hipSuccess) e2 = hipEventElapsedTime(&ms, o0, o1);
                    if (pass > 0) ms_mode[fused] = std::min(ms_mode[fused], ms);
                }
            }
            if (e2 != hipSuccess) break;
            for (int fused = 1; fused >= 0; --fused) {
                if (ms_mode[fused] < best_obs_ms) {
                    best_obs_ms = ms_mode[fused];
                    best_rows = rows;
                    best_kind = sh.kind;
                    best_k = sh.k;
                    best_fused = fused != 0;
                }
            }
        }
        if (o0) (void)hipEventDestroy(o0);
        if (o1) (void)hipEventDestroy(o1);
        c->obs_fusion = (e2 == hipSuccess) ? best_fused : true;
        c->rows_fused = (e2 == hipSuccess) ? best_rows : chosen_rows;
        c->fuse_kind = (e2 == hipSuccess) ? best_kind : chosen_kind;
        c->fuse_k = (e2 == hipSuccess) ? best_k : chosen_k;
        build_tiles(c, kFusedTiles, c->rows_fused);
        build_tiles(c, kStripTiles, c->rows_fused);
        if (e2 == hipSuccess) e2 = upload_tiles(c, kFusedTiles);
        if (e2 == hipSuccess) e2 = upload_tiles(c, kStripTiles);
        if (e2 == hipSuccess) e2 = launch_copy(c->prec, red, backup, psi, c->stream);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->stream);
    }
    c->timing = keep_timing;
    c->drop_graphs();
    if (e != hipSuccess) return c->hip_fail(e, "tdse_autotune_taylor");
    if (e2 != hipSuccess) return c->hip_fail(e2, "tdse_autotune_taylor restore");
    if (!bad.empty() && c->prec == TDSE_FP64)
        return c->fail(TDSE_E_HIP, "tdse_autotune_taylor: fused steps differ from the per-term step:" + bad);
    if (k_out) *k_out = c->fuse_k;
    if (rows_out) *rows_out = c->rows_fused;
    return TDSE_OK;
}

extern "C" int32_t tdse_taylor_fusion(const tdse_ctx* c) { return c ? c->fuse_k : 0; }
extern "C" int32_t tdse_taylor_fusion_kind(const tdse_ctx* c) { return c ? c->fuse_kind : 0; }

extern "C" tdse_status tdse_set_taylor_fusion(tdse_ctx* c, int32_t k, int32_t rows, int32_t kind)
{
    if (!c) return TDSE_E_INVALID;
    if (k < 0 || k > kMaxFused || (k > 0 && (rows < 1 || rows > 64)) || kind < 0 || kind > 3)
        return c->fail(TDSE_E_INVALID, "tdse_set_taylor_fusion: k must be 0..8, rows 1..64, kind 0..3");
    if (c->prec == TDSE_FP48 && k > 0 && kind == 0)
        return c->fail(TDSE_E_INVALID, "tdse_set_taylor_fusion: the LDS-ring kernel (kind 0) has no 48-bit form");
    if (c->bound) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "tdse_set_taylor_fusion sync");
    }
    // the tile regions hold the row-1 count of the narrowest tiles of either kind
    if (k > 0) c->rows_fused = rows;
    c->fuse_k = k;
    c->fuse_kind = kind;
    build_tiles(c, kFusedTiles, c->rows_fused);
    build_tiles(c, kStripTiles, c->rows_fused);
    if (c->tiles[kFusedTiles].size() > c->tile_cap[kFusedTiles] || c->tiles[kStripTiles].size() > c->tile_cap[kStripTiles])
        return c->fail(TDSE_E_INVALID, "tdse_set_taylor_fusion: tile table larger than its workspace region");
    if (c->bound) {
        hipError_t e = upload_tiles(c, kFusedTiles);
        if (e == hipSuccess) e = upload_tiles(c, kStripTiles);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "tdse_set_taylor_fusion upload");
    }
    c->drop_graphs();
    return TDSE_OK;
}

extern "C" tdse_status tdse_set_sweep_shape(tdse_ctx* c, int32_t rows, int32_t variant)
{
    if (!c) return TDSE_E_INVALID;
    if (rows < 1 || rows > kTileRows || variant < 0 || variant > 7)
        return c->fail(TDSE_E_INVALID, "tdse_set_sweep_shape: rows must be 1..32 and variant 0..7");
    if (c->prec == TDSE_FP48 && (variant & 5) == 1)
        return c->fail(TDSE_E_INVALID, "tdse_set_sweep_shape: two-radii sweeps have no 48-bit form");
    if (c->bound) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "tdse_set_sweep_shape sync");
    }
    c->rows_sweep = rows;
    c->sweep_variant = variant;
    build_tiles(c, kSweepTiles, rows);
    build_tiles(c, kPairTiles, rows);
    build_tiles(c, kApplyTiles, rows);
    if (c->bound) {
        hipError_t e = upload_tiles(c, kSweepTiles);
        if (e == hipSuccess) e = upload_tiles(c, kPairTiles);
        if (e == hipSuccess) e = upload_tiles(c, kApplyTiles);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "tdse_set_sweep_shape upload");
    }
    c->drop_graphs();
    return TDSE_OK;
}

extern "C" int32_t tdse_tile_rows(const tdse_ctx* c) { return c ? c->rows_sweep : 0; }
extern "C" int32_t tdse_sweep_variant(const tdse_ctx* c) { return c ? c->sweep_variant : 0; }

extern "C" tdse_status tdse_use_graphs(tdse_ctx* c, int32_t enable)
{
    if (!c) return TDSE_E_INVALID;
    if (c->bound) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "tdse_use_graphs sync");
    }
    c->use_graphs = enable != 0;
    if (!c->use_graphs) c->drop_graphs();
    return TDSE_OK;
}

extern "C" tdse_status tdse_set_rk4_fusion(tdse_ctx* c, int32_t enable)
{
    if (!c) return TDSE_E_INVALID;
    if (c->bound) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "tdse_set_rk4_fusion sync");
    }
    c->rk4_fused = enable != 0;
    c->drop_graphs();
    return TDSE_OK;
}

extern "C" int32_t tdse_rk4_fusion(const tdse_ctx* c) { return (c && c->rk4_fused) ? 1 : 0; }

extern "C" tdse_status tdse_set_obs_fusion(tdse_ctx* c, int32_t enable)
{
    if (!c) return TDSE_E_INVALID;
    if (c->bound) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess && c->obs_stream) e = hipStreamSynchronize(c->obs_stream);
        if (e != hipSuccess) return c->hip_fail(e, "tdse_set_obs_fusion sync");
    }
    c->obs_fusion = enable != 0;
    c->drop_graphs();
    return TDSE_OK;
}

extern "C" int32_t tdse_obs_fusion(const tdse_ctx* c) { return c && c->obs_fusion ? 1 : 0; }

extern "C" tdse_status tdse_set_obs_overlap(tdse_ctx* c, int32_t enable)
{
    if (!c) return TDSE_E_INVALID;
    if (c->bound) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e == hipSuccess && c->obs_stream) e = hipStreamSynchronize(c->obs_stream);
        if (e != hipSuccess) return c->hip_fail(e, "tdse_set_obs_overlap sync");
    }
    c->obs_overlap = enable != 0;
    c->drop_graphs();
    return TDSE_OK;
}

// ---------------------------------------------------------------------------
// timing
// ---------------------------------------------------------------------------
extern "C" tdse_status tdse_timing_enable(tdse_ctx* c, int32_t enable)
{
    if (!c) return TDSE_E_INVALID;
    if (c->bound) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "tdse_timing_enable sync");
    }
    c->timing = enable != 0;
    c->ev_used = 0;
    return TDSE_OK;
}

extern "C" tdse_status tdse_timing_read(tdse_ctx* c, const char* kernel, int64_t* launches, double* total_ms)
{
    if (!c || !kernel || !launches || !total_ms) return TDSE_E_INVALID;
    const int kind = timed_kind(kernel);
    if (kind < 0) return c->fail(TDSE_E_INVALID, "tdse_timing_read: unknown kernel family");
    if (c->bound) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return c->hip_fail(e, "tdse_timing_read sync");
    }
    int64_t cnt = 0;
    double tot = 0.0;
    for (size_t s = 0; s < c->ev_used; ++s) {
        if (c->ev_kind[s] != kind) continue;
        float ms = 0.0f;
        hipError_t e = hipEventElapsedTime(&ms, c->ev_pool[s].first, c->ev_pool[s].second);
        if (e != hipSuccess) return c->hip_fail(e, "hipEventElapsedTime");
        ++cnt;
        tot += ms;
    }
    *launches = cnt;
    *total_ms = tot;
    return TDSE_OK;
}
