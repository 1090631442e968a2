// C ABI of libsph (declared in include/sph.h): argument checking, derived
// constants, the workspace layout, the chunk maps and the stage sequences.
#include "sph.h"
#include "sph_host.h"
#include "sph_launch.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

using namespace sphx;

namespace {

thread_local std::string g_err;

sph_status fail(sph_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(SPH_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

enum Stage { ST_KEYS = 0, ST_SCAN, ST_SORT, ST_REORDER, ST_PACK, ST_DENSITY, ST_FORCE, ST_REDUCE,
             ST_SUB_FIRST, ST_SUB_PRESSURE, ST_SUB_SECOND, ST_SUB_DENSITY, ST_BUILD, ST_COUNT };
const char *kStageNames[ST_COUNT] = {"keys", "cell_scan", "radix_sort", "reorder",
                                     "pack", "density", "force", "reduce",
                                     "sub_first_half", "sub_pressure", "sub_second_half", "sub_density",
                                     "build"};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Wendland C2 normalisation: W(0) for support 2h.
double wendland_alpha(int dim, double h)
{
    const double pi = 3.14159265358979323846;
    return dim == 2 ? 7.0 / (4.0 * pi * h * h) : 21.0 / (16.0 * pi * h * h * h);
}

// Number density of the perfect lattice of spacing dx: sum over Z^d of W(|k| dx).
double lattice_number_density(int dim, double dx, double h)
{
    const double a = wendland_alpha(dim, h);
    const int K = (int)std::ceil(2.0 * h / dx) + 1;
    double s = 0.0;
    const int kz0 = dim == 3 ? -K : 0, kz1 = dim == 3 ? K : 0;
    for (int kz = kz0; kz <= kz1; ++kz)
        for (int ky = -K; ky <= K; ++ky)
            for (int kx = -K; kx <= K; ++kx) {
                const double r = dx * std::sqrt((double)(kx * kx + ky * ky + kz * kz));
                const double q = r / h;
                if (q >= 2.0) continue;
                const double t = 1.0 - 0.5 * q;
                s += a * t * t * t * t * (2.0 * q + 1.0);
            }
    return s;
}

// Grid of one instance: origin tank_lo - 3 dx, ceil((extent + 6 dx) / cs) cells.
void instance_grid(const sph_instance_desc &d, int dim, double dx, double cs, double lo[3],
                   int ncell[3])
{
#pragma clang fp contract(off)
    for (int a = 0; a < 3; ++a) {
        if (a < dim) {
            lo[a] = d.tank_lo[a] - 3.0 * dx;
            const double ext = (d.tank_hi[a] - d.tank_lo[a]) + 6.0 * dx;
            ncell[a] = (int)std::ceil(ext / cs);
            if (ncell[a] < 1) ncell[a] = 1;
        } else {
            lo[a] = 0.0;
            ncell[a] = 1;
        }
    }
}

}  // namespace

struct sph_ctx {
    sph_params p{};
    std::vector<sph_instance_desc> inst;
    SimConst sc{};
    std::vector<InstDev> idev;
    std::vector<Chunk> fmap, wmap;
    std::vector<Chunk> rmap;     // first reduction level over the per-chunk partials
    int64_t N = 0, Nw = 0, C = 0;
    int block = 256;
    int lcap = 96;
    int pref = 8;
    bool list_valid = false;  // the neighbour list matches the current sorted order
    bool mixed = false;
    bool dual = false;        // dual-criteria Riemann scheme
    bool skin = false;        // Verlet skin: the device decides when to rebuild
    bool host = false;        // SPH_POLICY_HOST: the step runs on the host
    std::unique_ptr<HostExec> hexec;
    // workspace layout (byte offsets)
    size_t ws_bytes = 0;
    size_t o_skey, o_rk0, o_rv0, o_rk1, o_rv1, o_hist, o_part, o_cnt, o_rec,
        o_wkey, o_wskey, o_partials, o_rmap, o_subpart, o_fmap, o_wmap, o_inst, o_flags, o_clampc, o_nlist,
        o_lcount, o_cpos, o_wcpos, o_drho, o_nsub, o_dtsub, o_nsubmax, o_subtot, o_gate, o_disp, o_xb;
    // state
    bool bound = false, primed = false, cells_built = false;
    sph_buffers buf{};
    Dev dev{};
    int64_t steps_done = 0;
    int64_t substeps_done = 0;   // dual scheme: sub-step loop iterations
    // graphs
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    // timing: events around the stages whose bit (1 << stage) is set
    bool timing = false;
    uint32_t timing_mask = 0;
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double stage_ms[ST_COUNT] = {0};
    int64_t stage_n[ST_COUNT] = {0};
};

namespace {

hipEvent_t take_event(sph_ctx *c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct StageTimer {
    sph_ctx *c;
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr;
    StageTimer(sph_ctx *c_, int st, hipStream_t s_, bool on) : c(c_), stage(st), s(s_)
    {
        if (on && ((c->timing_mask >> st) & 1u)) {
            a = take_event(c);
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~StageTimer()
    {
        if (!a) return;
        hipEvent_t b = take_event(c);
        if (!b) return;
        (void)hipEventRecord(b, s);
        c->pending.push_back({stage, a, b});
    }
};

void collect_times(sph_ctx *c)
{
    for (auto &r : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            c->stage_ms[r.stage] += ms;
            c->stage_n[r.stage] += 1;
        }
        c->pool.push_back(r.a);
        c->pool.push_back(r.b);
    }
    c->pending.clear();
}

// bytes of one fluid sweep record (two 4-vectors) and of one wall record
int rec_bytes(bool mixed) { return mixed ? 32 : 64; }
int wall_rec_bytes(int dim, bool mixed) { return mixed ? 16 : (dim == 3 ? 32 : 16); }

void build_layout(sph_ctx *c)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(std::max<size_t>(bytes, 1));
        return o;
    };
    const int64_t nmax = std::max<int64_t>(std::max<int64_t>(c->N, c->Nw), 1);
    const int dim = c->p.dim;
    c->o_skey = take(sizeof(int) * std::max<int64_t>(c->N, 1));
    c->o_rk0 = take(sizeof(int) * nmax);
    c->o_rv0 = take(sizeof(int) * nmax);
    c->o_rk1 = take(sizeof(int) * nmax);
    c->o_rv1 = take(sizeof(int) * nmax);
    c->o_hist = take(sizeof(int) * 256 * (size_t)radix_tiles(nmax));
    c->o_part = take(sizeof(int) * 16384);
    c->o_cnt = take(sizeof(int) * (c->C + 1));
    const size_t nf = (size_t)std::max<int64_t>(c->N, 1);
    // the sweep records share their memory with the reorder gather buffer:
    // the reorder runs before the records are packed
    const size_t scr_bytes = nf * sizeof(double) * (2 * dim + 2);
    // the wall records follow the fluid records (and the reorder buffer) in
    // one region, so that the list walks address both from one base; 64
    // bytes of padding at its end: a cooperative walk reads whole fluid-record
    // sizes, also at the last wall record
    const size_t wrec_off = align256(std::max(nf * rec_bytes(c->mixed), scr_bytes));
    c->sc.wrec_off = (int64_t)wrec_off;
    c->o_rec = take(wrec_off + (size_t)std::max<int64_t>(c->Nw, 1) * wall_rec_bytes(dim, c->mixed) + 64);
    c->o_wkey = take(sizeof(int) * std::max<int64_t>(c->Nw, 1));
    c->o_wskey = take(sizeof(int) * std::max<int64_t>(c->Nw, 1));
    c->o_partials = take(sizeof(double) * kNPart * std::max<size_t>(c->fmap.size(), 1));
    c->o_rmap = take(sizeof(Chunk) * std::max<size_t>(c->rmap.size(), 1));
    c->o_subpart = take(sizeof(double) * kNPart * std::max<size_t>(c->rmap.size(), 1));
    c->o_fmap = take(sizeof(Chunk) * std::max<size_t>(c->fmap.size(), 1));
    c->o_wmap = take(sizeof(Chunk) * std::max<size_t>(c->wmap.size(), 1));
    c->o_inst = take(sizeof(InstDev) * c->idev.size());
    c->o_flags = take(64);
    c->o_clampc = take(sizeof(int) * c->idev.size());
    c->o_lcount = take(sizeof(int) * nf);
    // FP32 cell-offset copies of the positions for the candidate tests
    const size_t cbytes = dim == 3 ? 16 : 8;
    c->o_cpos = take(nf * cbytes);
    c->o_wcpos = take((size_t)std::max<int64_t>(c->Nw, 1) * cbytes);
    c->o_nlist = take(c->lcap > 0 ? sizeof(unsigned) * nf * (size_t)c->lcap : 1);
    // dual scheme: continuity rates and the per-instance sub-step plan
    c->o_drho = take(c->dual ? sizeof(double) * nf : 1);
    c->o_nsub = take(sizeof(int) * c->idev.size());
    c->o_dtsub = take(sizeof(double) * c->idev.size());
    c->o_nsubmax = take(sizeof(int));
    c->o_subtot = take(sizeof(unsigned long long));
    // Verlet skin: rebuild / reorder gates, counters and displacement bounds
    c->o_gate = take(sizeof(int) * 8);
    c->o_disp = take(sizeof(double) * 2);
    c->o_xb = take(c->dual && c->skin ? sizeof(double) * dim * nf : 1);
    c->ws_bytes = off;
}

// Launch order of chunks: block b (dispatched to XCD b % kXcds) takes the
// next chunk of the contiguous share of its XCD.  A bijection for any count.
std::vector<Chunk> xcd_order(const std::vector<Chunk> &chunks)
{
    const int n = (int)chunks.size();
    std::vector<Chunk> out(chunks.size());
    std::vector<int> offset(kXcds + 1, 0);
    for (int x = 0; x < kXcds; ++x) {
        const int count = x < n ? (n - 1 - x) / kXcds + 1 : 0;
        offset[x + 1] = offset[x] + count;
    }
    for (int b = 0; b < n; ++b) out[b] = chunks[offset[b % kXcds] + b / kXcds];
    return out;
}

void build_maps(sph_ctx *c)
{
    c->fmap.clear();
    c->wmap.clear();
    int64_t fo = 0, wo = 0;
    for (size_t b = 0; b < c->inst.size(); ++b) {
        InstDev &I = c->idev[b];
        I.fluid_off = (int)fo;
        I.n_fluid = c->inst[b].n_fluid;
        I.wall_off = (int)wo;
        I.n_wall = c->inst[b].n_wall;
        I.chunk_begin = (int)c->fmap.size();
        for (int64_t s = fo; s < fo + I.n_fluid; s += c->block)
            c->fmap.push_back({(int)b, (int)s, (int)std::min<int64_t>(s + c->block, fo + I.n_fluid),
                               (int)c->fmap.size()});
        I.chunk_end = (int)c->fmap.size();
        for (int64_t s = wo; s < wo + I.n_wall; s += c->block)
            c->wmap.push_back({(int)b, (int)s, (int)std::min<int64_t>(s + c->block, wo + I.n_wall),
                               (int)c->wmap.size()});
        fo += I.n_fluid;
        wo += I.n_wall;
    }
    c->fmap = xcd_order(c->fmap);
    c->wmap = xcd_order(c->wmap);
    // the partial sums of an instance's chunks are reduced in two levels:
    // fixed runs of kReduceRows chunk rows per block, then the runs (a fixed
    // order, so the sums do not depend on scheduling)
    c->rmap.clear();
    for (size_t b = 0; b < c->inst.size(); ++b) {
        InstDev &I = c->idev[b];
        I.sub_begin = (int)c->rmap.size();
        for (int r = I.chunk_begin; r < I.chunk_end; r += kReduceRows)
            c->rmap.push_back({(int)b, r, std::min(r + kReduceRows, I.chunk_end), (int)c->rmap.size()});
        I.sub_end = (int)c->rmap.size();
    }
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

sph_status check_launch(hipError_t e, const char *what)
{
    if (e != hipSuccess) return fail(SPH_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return SPH_OK;
}

#define TRY(st)                         \
    do {                                \
        sph_status s_ = (st);           \
        if (s_ != SPH_OK) return s_;    \
    } while (0)

// ---- stage sequences ------------------------------------------------------

sph_status do_keys(sph_ctx *c, int kick_on, hipStream_t s, bool timed)
{
    StageTimer t(c, ST_KEYS, s, timed);
    return check_launch(launch_keys(c->sc, c->dev, kick_on, s), "keys");
}

sph_status do_sort(sph_ctx *c, bool reorder, hipStream_t s, bool timed, int kick_on = 0)
{
    const Dev &d = c->dev;
    c->list_valid = false;
    {
        StageTimer t(c, ST_SCAN, s, timed);
        TRY(check_launch(launch_exclusive_scan(d.cnt, d.cell_start, c->C + 1, d.part, 1, s, d.gate),
                         "cell scan"));
    }
    {
        StageTimer t(c, ST_SORT, s, timed);
        TRY(check_launch(launch_radix_sort(d.key, c->N, c->C, d.skey, d.perm, d.rk0, d.rv0, d.rk1,
                                           d.rv1, d.hist, d.part, s, d.gate),
                         "radix sort"));
    }
    if (reorder) {
        StageTimer t(c, ST_REORDER, s, timed);
        TRY(check_launch(launch_reorder(c->sc, d, s), "reorder"));
    }
    StageTimer t(c, ST_PACK, s, timed);
    return check_launch(launch_pack(c->sc, d, c->mixed, s, kick_on), "pack");
}

sph_status do_density(sph_ctx *c, int use_dt, hipStream_t s, bool timed)
{
    {
        StageTimer t(c, ST_BUILD, s, timed);
        TRY(check_launch(launch_build(c->sc, c->dev, c->mixed, s), "build"));
    }
    StageTimer t(c, ST_DENSITY, s, timed);
    c->list_valid = c->lcap > 0;
    return check_launch(launch_density(c->sc, c->dev, c->mixed, use_dt, s), "density");
}

sph_status do_force(sph_ctx *c, int fused, hipStream_t s, bool timed)
{
    StageTimer t(c, ST_FORCE, s, timed);
    const int list = c->lcap > 0 && c->list_valid;
    return check_launch(launch_force(c->sc, c->dev, c->mixed, fused, list, s), "force");
}

sph_status do_reduce(sph_ctx *c, int prime, hipStream_t s, bool timed)
{
    StageTimer t(c, ST_REDUCE, s, timed);
    return check_launch(launch_final_reduce(c->sc, c->dev, prime, s), "reduce");
}

bool reorder_due(const sph_ctx *c)
{
    // with a skin the reorder kernels are always enqueued and the device runs
    // them on a rebuild at least reorder_every steps after the last reorder
    if (c->skin) return c->p.reorder_every > 0;
    return c->p.reorder_every > 0 && (c->steps_done % c->p.reorder_every) == 0;
}

// The prime builds; its reduction (the first scheme) or the displacement
// check after it (the dual scheme) plans the first step.  The first rebuild
// after it reorders, as the first step does without a skin.
hipError_t skin_prime_gates(sph_ctx *c, hipStream_t s)
{
    const Dev &d = c->dev;
    const int K = c->p.reorder_every;
    hipError_t e = launch_fill_i32(d.gate, 8, 0, s);
    if (e == hipSuccess) e = launch_fill_i32(d.gate, 1, 1, s);
    if (e == hipSuccess) e = launch_fill_i32(d.gate + 2, 1, K > 0 ? K - 1 : 0, s);
    if (e == hipSuccess) e = launch_fill_f64(d.disp, 2, 0.0, s);
    return e;
}

// ---- dual-criteria scheme ------------------------------------------------

sph_status do_dual_part(sph_ctx *c, int sub, int part, hipStream_t s, bool timed)
{
    static const Stage stage[4] = {ST_SUB_FIRST, ST_SUB_PRESSURE, ST_SUB_SECOND, ST_SUB_DENSITY};
    const int list = c->lcap > 0 && c->list_valid;
    StageTimer t(c, stage[part], s, timed);
    return check_launch(launch_dual_substep(c->sc, c->dev, sub, list, s, part), "dual sub-step");
}

// State partials, then the per-instance reductions with the plan of the
// next advection step (and its maximum sub-step count).
sph_status dual_reduce(sph_ctx *c, int prime, hipStream_t s, bool timed)
{
    const Dev &d = c->dev;
    TRY(check_launch(launch_half2(c->sc, d, s, 0), "state partials"));
    TRY(check_launch(launch_fill_i32(d.nsub_max, 1, 0, s), "plan reset"));
    if (d.gate) TRY(check_launch(launch_skin_displacement(c->sc, d, s), "skin check"));
    return do_reduce(c, prime, s, timed);
}

// Step 0: cell table and summation at x0, pressure and the pressure sweep
// with dt = 0, reductions and the first plan.
sph_status dual_prime(sph_ctx *c, hipStream_t s)
{
    const Dev &d = c->dev;
    const int64_t B = (int64_t)c->idev.size();
    if (d.gate) TRY(check_launch(skin_prime_gates(c, s), "fill"));
    TRY(do_keys(c, 0, s, false));
    TRY(do_sort(c, false, s, false));
    if (d.gate) TRY(check_launch(launch_save_build_positions(c->sc, d, s), "build positions"));
    TRY(do_density(c, 0, s, false));
    TRY(check_launch(launch_fill_f64(d.drho, c->N, 0.0, s), "fill"));
    TRY(check_launch(launch_fill_i32(d.nsub, B, 1, s), "fill"));
    TRY(check_launch(launch_fill_f64(d.dtsub, B, 0.0, s), "fill"));
    TRY(check_launch(launch_fill_i32(reinterpret_cast<int *>(d.subs_total), 2, 0, s), "fill"));
    TRY(do_dual_part(c, 0, 0, s, false));
    TRY(do_dual_part(c, 0, 1, s, false));
    return dual_reduce(c, 1, s, false);
}

// One advection step: cell table, records and summation (with the list) at
// the current positions, then nsub_bound acoustic sub-step slots, of which
// each instance runs the ones its plan asks for (the kernels of a later slot
// return at once).  No host synchronisation: the step can be captured.
sph_status dual_advection_step(sph_ctx *c, bool reorder, hipStream_t s, bool timed)
{
    const Dev &d = c->dev;
    TRY(check_launch(launch_count_substeps(d, s), "sub-step count"));
    TRY(do_keys(c, 0, s, timed));
    TRY(do_sort(c, reorder, s, timed));
    if (d.gate) TRY(check_launch(launch_save_build_positions(c->sc, d, s), "build positions"));
    TRY(do_density(c, 0, s, timed));
    TRY(check_launch(launch_fill_f64(d.drho, c->N, 0.0, s), "fill"));
    for (int sub = 0; sub < c->sc.nsub_bound; ++sub)
        for (int part = 0; part < 4; ++part) TRY(do_dual_part(c, sub, part, s, timed));
    return dual_reduce(c, 0, s, timed);
}

sph_status enqueue_step(sph_ctx *c, bool reorder, hipStream_t s, bool timed)
{
    TRY(do_keys(c, 1, s, timed));
    TRY(do_sort(c, reorder, s, timed, 1));
    TRY(do_density(c, 1, s, timed));
    TRY(do_force(c, 1, s, timed));
    return do_reduce(c, 0, s, timed);
}

sph_status ensure_graph(sph_ctx *c, int variant)
{
    if (c->gexec[variant]) return SPH_OK;
    if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    sph_status st = c->dual ? dual_advection_step(c, variant == 1, c->cap_stream, false)
                            : enqueue_step(c, variant == 1, c->cap_stream, false);
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (st != SPH_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(SPH_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&c->gexec[variant], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->gexec[variant] = nullptr;
        return fail(SPH_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    return SPH_OK;
}

void drop_graphs(sph_ctx *c)
{
    for (auto &g : c->gexec)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

}  // namespace

// =========================================================================
// ABI
// =========================================================================

extern "C" {

const char *sph_last_error(void) { return g_err.c_str(); }

const char *sph_stage_name(int32_t stage)
{
    if (stage < 0 || stage >= ST_COUNT) return "";
    return kStageNames[stage];
}

int32_t sph_stage_count(void) { return ST_COUNT; }

sph_status sph_create(const sph_params *p, sph_ctx **out)
{
    if (!p || !out) return fail(SPH_E_ARG, "null argument");
    *out = nullptr;
    if (p->dim != 2 && p->dim != 3) return fail(SPH_E_ARG, "dim must be 2 or 3");
    if (p->precision != SPH_FP64 && p->precision != SPH_MIXED) return fail(SPH_E_ARG, "unknown precision");
    if (p->n_instances < 1 || !p->inst) return fail(SPH_E_ARG, "need at least one instance");
    if (p->reorder_every < 0) return fail(SPH_E_ARG, "reorder_every must be >= 0");
    if (!(p->dx > 0.0) || !(p->h > 0.0) || !(p->rho0 > 0.0)) return fail(SPH_E_ARG, "dx, h and rho0 must be positive");
    if (!(p->alpha >= 0.0) || !(p->eps > 0.0) || !(p->cfl_ac > 0.0) || !(p->cfl_f > 0.0))
        return fail(SPH_E_ARG, "alpha >= 0, eps > 0 and positive Courant numbers required");
    const int block = p->block_threads == 0 ? 256 : p->block_threads;
    if (block != 64 && block != 128 && block != 256) return fail(SPH_E_ARG, "block_threads must be 0, 64, 128 or 256");
    if (!(p->skin >= 0.0 && p->skin <= 2.0 * p->h)) return fail(SPH_E_ARG, "skin must be in [0, 2h]");
    // default capacity: the neighbours within 2h + skin, scaled from 2h
    const double grow = std::pow((2.0 * p->h + p->skin) / (2.0 * p->h), p->dim);
    int lcap = p->list_cap == 0 ? (int)std::ceil((p->dim == 3 ? 96 : 40) * grow)
                                : (p->list_cap < 0 ? 0 : p->list_cap);
    lcap = (lcap + 3) & ~3;   // stored in quads
    const int pref = p->prefetch == 0 ? 8 : p->prefetch;
    if (pref != 4 && pref != 8) return fail(SPH_E_ARG, "prefetch must be 0, 4 or 8");
    if (p->build < 0 || p->build > 2) return fail(SPH_E_ARG, "build must be 0, 1 or 2");
    if (lcap > 4096) return fail(SPH_E_ARG, "list_cap must be at most 4096");
    if (p->scheme != SPH_SCHEME_WCSPH && p->scheme != SPH_SCHEME_DUAL) return fail(SPH_E_ARG, "unknown scheme");
    if (p->key_order != SPH_KEYS_ROW_MAJOR && p->key_order != SPH_KEYS_MORTON_TILES)
        return fail(SPH_E_ARG, "unknown key order");
    if (p->policy != SPH_POLICY_DEVICE && p->policy != SPH_POLICY_HOST) return fail(SPH_E_ARG, "unknown policy");
    if (p->policy == SPH_POLICY_HOST) {
        if (p->precision != SPH_FP64) return fail(SPH_E_UNSUPPORTED, "the host policy runs in FP64 only");
        if (p->scheme != SPH_SCHEME_WCSPH) return fail(SPH_E_UNSUPPORTED, "the host policy runs the WCSPH scheme");
        if (p->skin != 0.0) return fail(SPH_E_UNSUPPORTED, "the host policy rebuilds the cells every step (skin = 0)");
        if (p->key_order != SPH_KEYS_ROW_MAJOR) return fail(SPH_E_UNSUPPORTED, "the host policy uses row-major keys");
        if (p->use_graph) return fail(SPH_E_UNSUPPORTED, "the host policy replays no graphs");
    }
    if (p->scheme == SPH_SCHEME_DUAL) {
        if (p->precision != SPH_FP64) return fail(SPH_E_UNSUPPORTED, "the dual scheme runs in FP64 only");
        if (!(p->cfl_adv > 0.0) || !(p->eta >= 0.0))
            return fail(SPH_E_ARG, "the dual scheme needs cfl_adv > 0 and eta >= 0");
    }
    auto *c = new sph_ctx();
    c->p = *p;
    c->p.inst = nullptr;
    c->block = block;
    c->lcap = lcap;
    c->pref = pref;
    c->mixed = p->precision == SPH_MIXED;
    c->dual = p->scheme == SPH_SCHEME_DUAL;
    c->skin = p->skin > 0.0;
    c->host = p->policy == SPH_POLICY_HOST;
    c->inst.assign(p->inst, p->inst + p->n_instances);
    const double cs = 2.0 * p->h + p->skin;
    int64_t N = 0, Nw = 0, C = 0;
    c->idev.resize(c->inst.size());
    for (size_t b = 0; b < c->inst.size(); ++b) {
        const sph_instance_desc &d = c->inst[b];
        if (d.n_fluid < 0 || d.n_wall < 0) { delete c; return fail(SPH_E_ARG, "negative particle count"); }
        if (!(d.c0 > 0.0)) { delete c; return fail(SPH_E_ARG, "c0 must be positive"); }
        for (int a = 0; a < p->dim; ++a)
            if (!(d.tank_hi[a] > d.tank_lo[a])) { delete c; return fail(SPH_E_ARG, "empty tank"); }
        InstDev &I = c->idev[b];
        std::memset(&I, 0, sizeof(I));
        instance_grid(d, p->dim, p->dx, cs, I.lo, I.ncell);
        // cells of the instance's key range (tiled Morton keys pad the grid to
        // whole tiles of 8^d cells)
        const int64_t nc = p->key_order == 0 ? (int64_t)I.ncell[0] * I.ncell[1] * I.ncell[2]
                                             : (int64_t)((I.ncell[0] + 7) / 8) * ((I.ncell[1] + 7) / 8) *
                                                   ((I.ncell[2] + 7) / 8) * (p->dim == 3 ? 512 : 64);
        I.cell_base = (int)std::min<int64_t>(C, INT32_MAX);
        I.c0 = d.c0;
        C += nc;
        N += d.n_fluid;
        Nw += d.n_wall;
    }
    if (N >= INT32_MAX || Nw >= INT32_MAX || C >= INT32_MAX - 1) { delete c; return fail(SPH_E_CAPACITY, "more than 2^31 particles or cells"); }
    if (C + 1 > scan_max_elems()) { delete c; return fail(SPH_E_CAPACITY, "too many cells for the two-level scan"); }
    if (lcap > 0 && (N >= (1 << 25) || Nw >= (1 << 25))) { delete c; return fail(SPH_E_CAPACITY, "the neighbour list addresses fewer than 2^25 particles per kind; use list_cap = -1"); }
    if ((int64_t)256 * radix_tiles(std::max(N, Nw)) > scan_max_elems()) { delete c; return fail(SPH_E_CAPACITY, "too many particles for the radix histogram scan"); }
    c->N = N;
    c->Nw = Nw;
    c->C = C;
    build_maps(c);
    // constants
    SimConst &sc = c->sc;
    sc.dim = p->dim;
    sc.n_inst = p->n_instances;
    sc.N = (int)N;
    sc.Nw = (int)Nw;
    sc.C = (int)C;
    sc.h = p->h;
    sc.inv_h = 1.0 / p->h;
    sc.cs = cs;
    sc.inv_cs = 1.0 / cs;
    sc.cut2 = (2.0 * p->h) * (2.0 * p->h);
    sc.bcut2 = cs * cs;
    sc.skin = p->skin;
    sc.reorder_every = p->reorder_every;
    sc.key_order = p->key_order;
    sc.rho0 = p->rho0;
    sc.sigma0 = lattice_number_density(p->dim, p->dx, p->h);
    sc.mass = p->rho0 / sc.sigma0;
    sc.alpha = p->alpha;
    sc.eps_h2 = p->eps * p->h * p->h;
    sc.cfl_ac = p->cfl_ac;
    sc.cfl_f = p->cfl_f;
    const double ka = wendland_alpha(p->dim, p->h);
    sc.kW = ka;
    sc.kF = -5.0 * ka / (p->h * p->h);
    sc.W0 = ka;
    for (int a = 0; a < 3; ++a) sc.g[a] = p->g[a];
    sc.scheme = c->dual ? 1 : 0;
    sc.cfl_adv = c->dual ? p->cfl_adv : 0.0;
    sc.cfl_sub = p->cfl_ac;
    sc.eta = c->dual ? p->eta : 0.0;
    // the plan's ceil(Dt / dac) = ceil(cfl_adv / cfl_ac * (c0 + vmax) / max(vmax,
    // c0 / 10)) peaks at vmax = c0 / 10, where the ratio is 11 cfl_adv / cfl_ac
    sc.nsub_bound = c->dual ? std::max(1, (int)std::ceil(11.0 * p->cfl_adv / p->cfl_ac * (1.0 + 1e-9))) : 1;
    if (c->dual && sc.nsub_bound > 4096) { delete c; return fail(SPH_E_ARG, "cfl_adv / cfl_ac plans more than 4096 sub-steps"); }
    sc.fh = (float)sc.h;
    sc.finv_h = (float)sc.inv_h;
    sc.fcs = (float)cs;
    sc.fcut2 = (float)sc.cut2;
    sc.fbcut2 = (float)sc.bcut2;
    sc.fkW = (float)sc.kW;
    sc.fkF = (float)sc.kF;
    sc.feps_h2 = (float)sc.eps_h2;
    for (int a = 0; a < 3; ++a) sc.fg[a] = (float)p->g[a];
    // mixed path: lengths in units of cs
    const double u2 = (2.0 * p->h) / cs;
    sc.ucut2 = (float)(u2 * u2);
    sc.ubcut2 = 1.0f;
    sc.uinv_h = (float)(cs / p->h);
    sc.ueps_h2 = (float)(p->eps * p->h * p->h / (cs * cs));
    for (int a = 0; a < 3; ++a) sc.ug[a] = (float)(p->g[a] * cs);
    sc.uvisc_scale = (float)(p->alpha * p->h / cs);
    sc.qcut2 = u2 * u2 * 0x1p62;
    sc.qbcut2 = 0x1p62;
    sc.qinv_h = cs / p->h * 0x1p-31;
    build_layout(c);
    // the list walks address fluid and padded wall records with 32-bit byte
    // offsets from one base
    if (c->host) c->ws_bytes = 0;   // the host executor keeps its scratch itself
    if (!c->host && lcap > 0 && (uint64_t)c->sc.wrec_off + (uint64_t)std::max<int64_t>(Nw, 1) * wall_rec_bytes(p->dim, c->mixed) + 64 >= (1ull << 32)) {
        delete c;
        return fail(SPH_E_CAPACITY, "the neighbour-list walks address at most 4 GiB of sweep records; use list_cap = -1");
    }
    *out = c;
    g_err.clear();
    return SPH_OK;
}

void sph_destroy(sph_ctx *ctx)
{
    if (!ctx) return;
    drop_graphs(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (auto &r : ctx->pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    delete ctx;
}

sph_status sph_get_info(const sph_ctx *ctx, sph_info *info)
{
    if (!ctx || !info) return fail(SPH_E_ARG, "null argument");
    info->n_fluid = ctx->N;
    info->n_wall = ctx->Nw;
    info->n_cells = ctx->C;
    info->workspace_bytes = ctx->ws_bytes;
    info->sigma0 = ctx->sc.sigma0;
    info->mass = ctx->sc.mass;
    info->cell_size = ctx->sc.cs;
    info->steps_done = ctx->steps_done;
    info->substeps_done = ctx->substeps_done;
    if (ctx->dual && ctx->primed) {
        // counted on the device (the plan never reaches the host)
        unsigned long long tot = 0;
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemcpy(&tot, ctx->dev.subs_total, sizeof(tot), hipMemcpyDeviceToHost));
        info->substeps_done = (int64_t)tot;
    }
    return SPH_OK;
}

sph_status sph_get_grid(const sph_ctx *ctx, int32_t b, double lo[3], int32_t ncell[3], int32_t *cell_base)
{
    if (!ctx || !lo || !ncell || !cell_base) return fail(SPH_E_ARG, "null argument");
    if (b < 0 || b >= (int32_t)ctx->idev.size()) return fail(SPH_E_ARG, "instance out of range");
    const InstDev &I = ctx->idev[b];
    for (int a = 0; a < 3; ++a) {
        lo[a] = I.lo[a];
        ncell[a] = I.ncell[a];
    }
    *cell_base = I.cell_base;
    return SPH_OK;
}

sph_status sph_workspace_size(const sph_ctx *ctx, size_t *bytes)
{
    if (!ctx || !bytes) return fail(SPH_E_ARG, "null argument");
    *bytes = ctx->ws_bytes;
    return SPH_OK;
}

sph_status sph_bind(sph_ctx *c, const sph_buffers *b, void *stream)
{
    if (!c || !b) return fail(SPH_E_ARG, "null argument");
    hipStream_t s = as_stream(stream);
    if (c->N > 0 && (!b->x || !b->v || !b->a || !b->rho || !b->id || !b->key || !b->perm || !b->count))
        return fail(SPH_E_ARG, "missing fluid buffer");
    if (c->Nw > 0 && (!b->xw || !b->wall_perm)) return fail(SPH_E_ARG, "missing wall buffer");
    if (c->host) {
        if (!b->cell_start || !b->wall_start || !b->dt || !b->diag)
            return fail(SPH_E_ARG, "missing table or per-instance buffer");
        int nt = (int)std::thread::hardware_concurrency();
        if (const char *e = std::getenv("SPH_HOST_THREADS")) nt = std::atoi(e);
        c->hexec.reset(new HostExec(c->sc, c->idev, c->p.reorder_every, nt > 0 ? nt : 1));
        c->buf = *b;
        c->hexec->bind(*b);
        c->bound = true;
        c->primed = false;
        c->cells_built = false;
        c->steps_done = 0;
        c->substeps_done = 0;
        return SPH_OK;
    }
    if (!b->cell_start || !b->wall_start || !b->dt || !b->diag || !b->workspace)
        return fail(SPH_E_ARG, "missing table, per-instance or workspace buffer");
    if (reinterpret_cast<uintptr_t>(b->workspace) % 256 != 0) return fail(SPH_E_ARG, "workspace must be 256-byte aligned");
    drop_graphs(c);
    c->buf = *b;
    char *ws = static_cast<char *>(b->workspace);
    Dev &d = c->dev;
    d.x = b->x; d.v = b->v; d.a = b->a; d.rho = b->rho;
    d.id = b->id; d.key = b->key; d.perm = b->perm; d.count = b->count;
    d.xw = b->xw; d.wall_perm = b->wall_perm; d.cell_start = b->cell_start; d.wall_start = b->wall_start;
    d.dt = b->dt; d.diag = b->diag;
    d.skey = reinterpret_cast<int *>(ws + c->o_skey);
    d.rk0 = reinterpret_cast<int *>(ws + c->o_rk0);
    d.rv0 = reinterpret_cast<int *>(ws + c->o_rv0);
    d.rk1 = reinterpret_cast<int *>(ws + c->o_rk1);
    d.rv1 = reinterpret_cast<int *>(ws + c->o_rv1);
    d.hist = reinterpret_cast<int *>(ws + c->o_hist);
    d.part = reinterpret_cast<int *>(ws + c->o_part);
    d.cnt = reinterpret_cast<int *>(ws + c->o_cnt);
    d.rec = ws + c->o_rec;
    d.scratch = reinterpret_cast<double *>(ws + c->o_rec);
    d.wpos = ws + c->o_rec + c->sc.wrec_off;
    d.cpos = ws + c->o_cpos;
    d.wcpos = ws + c->o_wcpos;
    d.wkey = reinterpret_cast<int *>(ws + c->o_wkey);
    d.wskey = reinterpret_cast<int *>(ws + c->o_wskey);
    d.partials = reinterpret_cast<double *>(ws + c->o_partials);
    d.rmap = reinterpret_cast<Chunk *>(ws + c->o_rmap);
    d.subpart = reinterpret_cast<double *>(ws + c->o_subpart);
    d.nrblocks = (int)c->rmap.size();
    d.fmap = reinterpret_cast<Chunk *>(ws + c->o_fmap);
    d.wmap = reinterpret_cast<Chunk *>(ws + c->o_wmap);
    d.inst = reinterpret_cast<InstDev *>(ws + c->o_inst);
    d.flags = reinterpret_cast<unsigned *>(ws + c->o_flags);
    d.clampc = reinterpret_cast<int *>(ws + c->o_clampc);
    d.nfchunks = (int)c->fmap.size();
    d.nwchunks = (int)c->wmap.size();
    d.block = c->block;
    d.list_cap = c->lcap;
    d.prefetch = c->pref;
    // cell pairs pay in 3D (about 18 targets per cell); in 2D (about 7) the
    // per-cell set-up outweighs them
    d.cell_pair = c->p.build == 2 || (c->p.build == 0 && c->p.dim == 3);
    d.nlist = reinterpret_cast<uint4 *>(ws + c->o_nlist);
    d.lcount = reinterpret_cast<int *>(ws + c->o_lcount);
    d.drho = reinterpret_cast<double *>(ws + c->o_drho);
    d.nsub = reinterpret_cast<int *>(ws + c->o_nsub);
    d.dtsub = reinterpret_cast<double *>(ws + c->o_dtsub);
    d.nsub_max = reinterpret_cast<int *>(ws + c->o_nsubmax);
    d.subs_total = reinterpret_cast<unsigned long long *>(ws + c->o_subtot);
    d.gate = c->skin ? reinterpret_cast<int *>(ws + c->o_gate) : nullptr;
    d.disp = c->skin ? reinterpret_cast<double *>(ws + c->o_disp) : nullptr;
    d.xb = c->dual && c->skin ? reinterpret_cast<double *>(ws + c->o_xb) : nullptr;
    if (!c->fmap.empty())
        HIP_TRY(hipMemcpyAsync(d.fmap, c->fmap.data(), sizeof(Chunk) * c->fmap.size(), hipMemcpyHostToDevice, s));
    if (!c->wmap.empty())
        HIP_TRY(hipMemcpyAsync(d.wmap, c->wmap.data(), sizeof(Chunk) * c->wmap.size(), hipMemcpyHostToDevice, s));
    if (!c->rmap.empty())
        HIP_TRY(hipMemcpyAsync(d.rmap, c->rmap.data(), sizeof(Chunk) * c->rmap.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d.inst, c->idev.data(), sizeof(InstDev) * c->idev.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_fill_i32(d.cnt, c->C + 1, 0, s));
    HIP_TRY(launch_fill_i32(reinterpret_cast<int *>(d.flags), 16, 0, s));
    HIP_TRY(launch_fill_i32(d.clampc, (int64_t)c->idev.size(), 0, s));
    // static wall table
    HIP_TRY(launch_wall_keys(c->sc, d, s));
    HIP_TRY(launch_exclusive_scan(d.cnt, d.wall_start, c->C + 1, d.part, 1, s));
    HIP_TRY(launch_radix_sort(d.wkey, c->Nw, c->C, d.wskey, d.wall_perm, d.rk0, d.rv0, d.rk1, d.rv1,
                              d.hist, d.part, s));
    HIP_TRY(launch_wall_pack(c->sc, d, c->mixed, s));
    HIP_TRY(launch_fill_i32(d.clampc, (int64_t)c->idev.size(), 0, s));
    HIP_TRY(hipStreamSynchronize(s));
    c->bound = true;
    c->primed = false;
    c->cells_built = false;
    c->list_valid = false;
    c->steps_done = 0;
    c->substeps_done = 0;
    return SPH_OK;
}

// Workspace owned by the library for callers that cannot allocate device
// memory (sph_bind_static).  Each device that loads the library holds its own
// copy until the process ends.  In host code the name stands for a host-side
// shadow, not for device memory: only the address that hipGetSymbolAddress
// returns for the current device is ever handed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[SPH_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
sph_status static_scratch_address(void **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SPH_E_UNSUPPORTED, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(SPH_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SPH_OK;
}

}  // namespace

sph_status sph_bind_static(sph_ctx *c, const sph_buffers *b, void *stream)
{
    if (c && c->host) return fail(SPH_E_UNSUPPORTED, "the host policy takes no device scratch");
    if (!c || !b) return fail(SPH_E_ARG, "null argument");
    if (c->ws_bytes > (size_t)SPH_STATIC_SCRATCH_BYTES)
        return fail(SPH_E_CAPACITY, "workspace of " + std::to_string(c->ws_bytes) +
                                        " bytes exceeds the static scratch of " +
                                        std::to_string((size_t)SPH_STATIC_SCRATCH_BYTES) +
                                        " bytes; use sph_bind with a caller workspace");
    void *ws = nullptr;
    const sph_status st = static_scratch_address(&ws);
    if (st != SPH_OK) return st;
    sph_buffers bb = *b;
    bb.workspace = ws;
    return sph_bind(c, &bb, stream);
}

sph_status sph_prime(sph_ctx *c, void *stream)
{
    if (!c) return fail(SPH_E_ARG, "null context");
    if (!c->bound) return fail(SPH_E_STATE, "sph_bind first");
    if (c->host) {
        c->hexec->prime();
        c->primed = true;
        c->steps_done = 0;
        return SPH_OK;
    }
    hipStream_t s = as_stream(stream);
    const Dev &d = c->dev;
    HIP_TRY(launch_fill_f64(d.diag, (int64_t)c->idev.size() * SPH_NDIAG, 0.0, s));
    HIP_TRY(launch_fill_i32(d.cnt, c->C + 1, 0, s));
    if (c->dual) {
        TRY(dual_prime(c, s));
    } else {
        if (c->skin) HIP_TRY(skin_prime_gates(c, s));
        TRY(do_keys(c, 0, s, false));
        TRY(do_sort(c, false, s, false));
        TRY(do_density(c, 0, s, false));
        TRY(do_force(c, 0, s, false));
        TRY(check_launch(launch_half2(c->sc, d, s, 0), "state partials"));
        TRY(do_reduce(c, 1, s, false));
    }
    c->primed = true;
    c->cells_built = false;
    c->steps_done = 0;
    c->substeps_done = 0;
    return SPH_OK;
}

sph_status sph_build_cells(sph_ctx *c, void *stream)
{
    if (!c) return fail(SPH_E_ARG, "null context");
    if (!c->bound) return fail(SPH_E_STATE, "sph_bind first");
    if (c->host) return fail(SPH_E_UNSUPPORTED, "the host policy runs whole steps (sph_step_batched)");
    if (c->dual) return fail(SPH_E_UNSUPPORTED, "stage calls are for the WCSPH scheme");
    if (c->skin) return fail(SPH_E_UNSUPPORTED, "stage calls rebuild every step: use skin = 0");
    if (c->cells_built) return fail(SPH_E_STATE, "cells already built: call sph_sort first");
    TRY(do_keys(c, 0, as_stream(stream), c->timing));
    c->cells_built = true;
    return SPH_OK;
}

sph_status sph_sort(sph_ctx *c, int32_t reorder, void *stream)
{
    if (!c) return fail(SPH_E_ARG, "null context");
    if (!c->bound) return fail(SPH_E_STATE, "sph_bind first");
    if (c->host) return fail(SPH_E_UNSUPPORTED, "the host policy runs whole steps (sph_step_batched)");
    if (c->dual) return fail(SPH_E_UNSUPPORTED, "stage calls are for the WCSPH scheme");
    if (c->skin) return fail(SPH_E_UNSUPPORTED, "stage calls rebuild every step: use skin = 0");
    if (!c->cells_built) return fail(SPH_E_STATE, "sph_build_cells (or sph_integrate half 1) first");
    TRY(do_sort(c, reorder != 0, as_stream(stream), c->timing));
    c->cells_built = false;
    return SPH_OK;
}

sph_status sph_density(sph_ctx *c, void *stream)
{
    if (!c) return fail(SPH_E_ARG, "null context");
    if (!c->bound) return fail(SPH_E_STATE, "sph_bind first");
    if (c->host) return fail(SPH_E_UNSUPPORTED, "the host policy runs whole steps (sph_step_batched)");
    if (c->dual) return fail(SPH_E_UNSUPPORTED, "stage calls are for the WCSPH scheme");
    if (c->skin) return fail(SPH_E_UNSUPPORTED, "stage calls rebuild every step: use skin = 0");
    return do_density(c, 1, as_stream(stream), c->timing);
}

sph_status sph_forces(sph_ctx *c, void *stream)
{
    if (!c) return fail(SPH_E_ARG, "null context");
    if (!c->bound) return fail(SPH_E_STATE, "sph_bind first");
    if (c->host) return fail(SPH_E_UNSUPPORTED, "the host policy runs whole steps (sph_step_batched)");
    if (c->dual) return fail(SPH_E_UNSUPPORTED, "stage calls are for the WCSPH scheme");
    if (c->skin) return fail(SPH_E_UNSUPPORTED, "stage calls rebuild every step: use skin = 0");
    return do_force(c, 0, as_stream(stream), c->timing);
}

sph_status sph_integrate(sph_ctx *c, int32_t half, void *stream)
{
    if (!c) return fail(SPH_E_ARG, "null context");
    if (!c->bound) return fail(SPH_E_STATE, "sph_bind first");
    if (c->host) return fail(SPH_E_UNSUPPORTED, "the host policy runs whole steps (sph_step_batched)");
    if (c->dual) return fail(SPH_E_UNSUPPORTED, "stage calls are for the WCSPH scheme");
    if (c->skin) return fail(SPH_E_UNSUPPORTED, "stage calls rebuild every step: use skin = 0");
    if (half != 1 && half != 2) return fail(SPH_E_ARG, "half must be 1 or 2");
    hipStream_t s = as_stream(stream);
    if (half == 1) {
        if (c->cells_built) return fail(SPH_E_STATE, "cells already built: call sph_sort first");
        TRY(do_keys(c, 1, s, c->timing));
        c->cells_built = true;
        return SPH_OK;
    }
    TRY(check_launch(launch_half2(c->sc, c->dev, s, 1), "half 2"));
    TRY(do_reduce(c, 0, s, c->timing));
    c->steps_done += 1;
    return SPH_OK;
}

sph_status sph_step_batched(sph_ctx *c, int32_t n_steps, void *stream)
{
    if (!c) return fail(SPH_E_ARG, "null context");
    if (n_steps < 0) return fail(SPH_E_ARG, "n_steps must be >= 0");
    if (!c->bound || !c->primed) return fail(SPH_E_STATE, "sph_bind and sph_prime first");
    if (c->cells_built) return fail(SPH_E_STATE, "a staged step is half done");
    if (c->host) {
        for (int32_t it = 0; it < n_steps; ++it) {
            c->hexec->step();
            c->steps_done += 1;
        }
        return SPH_OK;
    }
    hipStream_t s = as_stream(stream);
    const bool graph = c->p.use_graph && !c->timing;
    for (int32_t it = 0; it < n_steps; ++it) {
        const bool ro = reorder_due(c);
        if (graph) {
            TRY(ensure_graph(c, ro ? 1 : 0));
            HIP_TRY(hipGraphLaunch(c->gexec[ro ? 1 : 0], s));
        } else if (c->dual) {
            TRY(dual_advection_step(c, ro, s, c->timing));
        } else {
            TRY(enqueue_step(c, ro, s, c->timing));
        }
        c->steps_done += 1;
    }
    return SPH_OK;
}

sph_status sph_substeps(sph_ctx *c, int32_t *n, void *stream)
{
    if (!c || !n) return fail(SPH_E_ARG, "null argument");
    if (!c->dual) return fail(SPH_E_UNSUPPORTED, "sub-steps belong to the dual scheme");
    if (!c->bound || !c->primed) return fail(SPH_E_STATE, "sph_bind and sph_prime first");
    hipStream_t s = as_stream(stream);
    HIP_TRY(hipMemcpyAsync(n, c->dev.nsub, sizeof(int32_t) * c->idev.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SPH_OK;
}

sph_status sph_cell_builds(sph_ctx *c, int64_t *n, void *stream)
{
    if (!c || !n) return fail(SPH_E_ARG, "null argument");
    if (!c->bound || !c->primed) return fail(SPH_E_STATE, "sph_bind and sph_prime first");
    if (!c->skin) {
        *n = c->steps_done + 1;
        return SPH_OK;
    }
    hipStream_t s = as_stream(stream);
    int32_t host[8] = {0};
    HIP_TRY(hipMemcpyAsync(host, c->dev.gate, sizeof(host), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n = host[4];
    return SPH_OK;
}

sph_status sph_poll_errors(sph_ctx *c, uint32_t *flags, void *stream)
{
    if (!c || !flags) return fail(SPH_E_ARG, "null argument");
    if (!c->bound) return fail(SPH_E_STATE, "sph_bind first");
    if (c->host) {
        *flags = c->hexec->flags();
        c->hexec->clear_flags();
        return SPH_OK;
    }
    hipStream_t s = as_stream(stream);
    unsigned host = 0;
    HIP_TRY(hipMemcpyAsync(&host, c->dev.flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(launch_fill_i32(reinterpret_cast<int *>(c->dev.flags), 1, 0, s));
    HIP_TRY(hipStreamSynchronize(s));
    *flags = host;
    return SPH_OK;
}

sph_status sph_set_timing_mask(sph_ctx *c, uint32_t mask)
{
    if (!c) return fail(SPH_E_ARG, "null context");
    if (c->host && mask) return fail(SPH_E_UNSUPPORTED, "HIP events time the device policy only");
    c->timing_mask = mask & ((1u << ST_COUNT) - 1u);
    c->timing = c->timing_mask != 0;
    return SPH_OK;
}

sph_status sph_set_timing(sph_ctx *c, int32_t enable)
{
    if (!c) return fail(SPH_E_ARG, "null context");
    if (c->host && enable) return fail(SPH_E_UNSUPPORTED, "HIP events time the device policy only");
    c->timing = enable != 0;
    c->timing_mask = enable != 0 ? (1u << ST_COUNT) - 1u : 0u;
    return SPH_OK;
}

sph_status sph_stage_times(sph_ctx *c, double *ms, int64_t *launches, int32_t n, int32_t reset, void *stream)
{
    if (!c) return fail(SPH_E_ARG, "null context");
    if (c->host) return fail(SPH_E_UNSUPPORTED, "HIP events time the device policy only");
    HIP_TRY(hipStreamSynchronize(as_stream(stream)));
    collect_times(c);
    for (int32_t i = 0; i < n && i < ST_COUNT; ++i) {
        if (ms) ms[i] = c->stage_ms[i];
        if (launches) launches[i] = c->stage_n[i];
    }
    if (reset) {
        for (int i = 0; i < ST_COUNT; ++i) {
            c->stage_ms[i] = 0.0;
            c->stage_n[i] = 0;
        }
    }
    return SPH_OK;
}

}  // extern "C"
