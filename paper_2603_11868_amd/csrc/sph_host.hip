// Host execution of the WCSPH step (SPH_POLICY_HOST).  The arithmetic is the
// one of the GPU kernels, taken from sph_bodies.h; the loops around it are
// plain host loops over chunks of 4096 particles spread over std::threads.
// Every chunk is processed by one thread in slot order and its partial sums
// are combined in chunk order, so results do not depend on the thread count.
#include "sph_host.h"

#include <algorithm>
#include <atomic>
#include <thread>

#include "sph_bodies.h"

namespace sphx {

namespace {

constexpr int64_t kHostChunk = 4096;

struct HostChunk {
    int b;
    int64_t begin, end;
};

std::vector<HostChunk> host_chunks(const std::vector<int64_t> &fo)
{
    std::vector<HostChunk> out;
    for (int b = 0; b + 1 < (int)fo.size(); ++b)
        for (int64_t k = fo[b]; k < fo[b + 1]; k += kHostChunk)
            out.push_back({b, k, std::min(fo[b + 1], k + kHostChunk)});
    return out;
}

// f(chunk index) for every chunk, on up to nthreads threads.
template <class F>
void parallel_chunks(int64_t nchunks, int nthreads, F &&f)
{
    if (nchunks <= 0) return;
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(nthreads, nchunks));
    if (T == 1) {
        for (int64_t c = 0; c < nchunks; ++c) f(c);
        return;
    }
    std::atomic<int64_t> next{0};
    auto work = [&]() {
        for (int64_t c = next++; c < nchunks; c = next++) f(c);
    };
    std::vector<std::thread> pool;
    pool.reserve(T - 1);
    for (int t = 1; t < T; ++t) pool.emplace_back(work);
    work();
    for (auto &th : pool) th.join();
}

}  // namespace

HostExec::HostExec(const SimConst &sc, const std::vector<InstDev> &inst, int reorder_every, int nthreads)
    : sc_(sc), inst_(inst), K_(reorder_every), nthreads_(nthreads > 0 ? nthreads : 1)
{
    fo_.assign(inst.size() + 1, 0);
    for (size_t b = 0; b < inst.size(); ++b) fo_[b + 1] = fo_[b] + inst[b].n_fluid;
    N_ = sc.N;
    Nw_ = sc.Nw;
    C_ = sc.C;
}

void HostExec::bind(const sph_buffers &b)
{
    buf_ = b;
    const int dim = sc_.dim;
    skey_.assign(N_, 0);
    cnt_.assign(C_ + 1, 0);
    clamped_.assign(inst_.size(), 0);
    xs_.assign((size_t)dim * N_, 0.0);
    vs_.assign((size_t)dim * N_, 0.0);
    rhos_.assign(N_, 0.0);
    Ps_.assign(N_, 0.0);
    // the static wall table: keys, stable counting sort, sorted positions
    wkey_.assign(Nw_, 0);
    std::vector<int> wcnt(C_ + 1, 0);
    int64_t w0 = 0;
    for (size_t bi = 0; bi < inst_.size(); ++bi) {
        const InstDev &I = inst_[bi];
        for (int64_t w = w0; w < w0 + I.n_wall; ++w) {
            int cc[3] = {0, 0, 0}, cl = 0;
            for (int c = 0; c < dim; ++c) cc[c] = cell_1d(b.xw[c * Nw_ + w], I.lo[c], sc_.inv_cs, I.ncell[c], cl);
            const int k = I.cell_base + cell_key(sc_, I, cc[0], cc[1], cc[2]);
            wkey_[w] = k;
            ++wcnt[k];
        }
        w0 += I.n_wall;
    }
    int acc = 0;
    for (int64_t c = 0; c <= C_; ++c) {
        b.wall_start[c] = acc;
        acc += c < C_ ? wcnt[c] : 0;
    }
    std::vector<int> cur(b.wall_start, b.wall_start + C_);
    xws_.assign((size_t)dim * std::max<int64_t>(Nw_, 1), 0.0);
    for (int64_t w = 0; w < Nw_; ++w) {
        const int s = cur[wkey_[w]]++;
        b.wall_perm[s] = (int)w;
        for (int c = 0; c < dim; ++c) xws_[c * Nw_ + s] = b.xw[c * Nw_ + w];
    }
    flags_ = 0;
    steps_ = 0;
}

// Half 1 (optional) and the cell key of every particle, with the per-cell counts.
template <int DIM>
void HostExec::keys(bool kick_on)
{
    const auto chunks = host_chunks(fo_);
    std::vector<int> clamp(chunks.size(), 0);
    double *x = buf_.x, *v = buf_.v;
    const double *a = buf_.a;
    const int64_t n = N_;
    parallel_chunks((int64_t)chunks.size(), nthreads_, [&](int64_t ci) {
        const HostChunk &hc = chunks[ci];
        const InstDev &I = inst_[hc.b];
        const double dtb = buf_.dt[hc.b];
        for (int64_t i = hc.begin; i < hc.end; ++i) {
            double xi[3] = {0, 0, 0};
            for (int c = 0; c < DIM; ++c) {
                xi[c] = x[c * n + i];
                if (kick_on) {
                    double vc = v[c * n + i];
                    kick_drift(xi[c], vc, a[c * n + i], dtb);
                    v[c * n + i] = vc;
                    x[c * n + i] = xi[c];
                }
            }
            int cc[3] = {0, 0, 0}, cl = 0;
            for (int c = 0; c < DIM; ++c) cc[c] = cell_1d(xi[c], I.lo[c], sc_.inv_cs, I.ncell[c], cl);
            buf_.key[i] = I.cell_base + cell_key(sc_, I, cc[0], cc[1], cc[2]);
            clamp[ci] += cl;
        }
    });
    for (size_t ci = 0; ci < chunks.size(); ++ci) {
        clamped_[chunks[ci].b] += clamp[ci];
        if (clamp[ci]) flags_ |= SPH_FLAG_CLAMPED;
    }
}

// Stable counting sort of the storage slots by key (the definition of the
// sorted order), the cell start table, and the physical reorder when due.
void HostExec::sort(bool reorder)
{
    std::fill(cnt_.begin(), cnt_.end(), 0);
    for (int64_t i = 0; i < N_; ++i) ++cnt_[buf_.key[i]];
    int acc = 0;
    for (int64_t c = 0; c <= C_; ++c) {
        buf_.cell_start[c] = acc;
        acc += c < C_ ? cnt_[c] : 0;
    }
    std::vector<int> cur(buf_.cell_start, buf_.cell_start + C_);
    for (int64_t i = 0; i < N_; ++i) {
        const int s = cur[buf_.key[i]]++;
        buf_.perm[s] = (int)i;
        skey_[s] = buf_.key[i];
    }
    if (!reorder) return;
    // arrays gathered into sorted order; the accelerations are rewritten by
    // the force sweep of the step
    const int dim = sc_.dim;
    const int64_t n = N_;
    std::vector<double> xt((size_t)dim * n), vt((size_t)dim * n), rt(n);
    std::vector<int> it(n);
    for (int64_t k = 0; k < n; ++k) {
        const int i = buf_.perm[k];
        for (int c = 0; c < dim; ++c) {
            xt[c * n + k] = buf_.x[c * n + i];
            vt[c * n + k] = buf_.v[c * n + i];
        }
        rt[k] = buf_.rho[i];
        it[k] = buf_.id[i];
    }
    std::copy(xt.begin(), xt.end(), buf_.x);
    std::copy(vt.begin(), vt.end(), buf_.v);
    std::copy(rt.begin(), rt.end(), buf_.rho);
    std::copy(it.begin(), it.end(), buf_.id);
    for (int64_t k = 0; k < n; ++k) {
        buf_.perm[k] = (int)k;
        buf_.key[k] = skey_[k];
    }
}

// Sorted copies of the sources' positions and velocities.
template <int DIM>
void HostExec::pack()
{
    const int64_t n = N_;
    const auto chunks = host_chunks(fo_);
    parallel_chunks((int64_t)chunks.size(), nthreads_, [&](int64_t ci) {
        for (int64_t k = chunks[ci].begin; k < chunks[ci].end; ++k) {
            const int i = buf_.perm[k];
            for (int c = 0; c < DIM; ++c) {
                xs_[c * n + k] = buf_.x[c * n + i];
                vs_[c * n + k] = buf_.v[c * n + i];
            }
        }
    });
}

// Sources of target k in the order of the direct search: stencil rows in z,
// y order; per row the fluid slots of its (up to) three cells in x order, then
// their wall slots.  fn(wall, s, r, r2) for every source closer than 2h.
template <int DIM, class Fn>
static void host_neighbours(const SimConst &sc, const InstDev &I, int lk, int64_t k, const double *pi,
                            const int *cstart, const int *wstart, const double *xs, int64_t n, const double *xws,
                            int64_t nw, Fn &&fn)
{
    int cx, cy, cz;
    cell_coords(sc, I, lk, cx, cy, cz);
    const int dz0 = (DIM == 3 && cz > 0) ? -1 : 0, dz1 = (DIM == 3 && cz < I.ncell[2] - 1) ? 1 : 0;
    const int xlo = cx > 0 ? cx - 1 : cx, xhi = cx < I.ncell[0] - 1 ? cx + 1 : cx;
    for (int dz = dz0; dz <= dz1; ++dz) {
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = cy + dy;
            if (yy < 0 || yy >= I.ncell[1]) continue;
            for (int pass = 0; pass < 2; ++pass) {
                const int *st = pass == 0 ? cstart : wstart;
                const double *src = pass == 0 ? xs : xws;
                const int64_t ns = pass == 0 ? n : nw;
                for (int xx = xlo; xx <= xhi; ++xx) {
                    const int key = I.cell_base + cell_key(sc, I, xx, yy, cz + dz);
                    for (int s = st[key]; s < st[key + 1]; ++s) {
                        if (pass == 0 && s == k) continue;
                        double r[3] = {0, 0, 0};
                        for (int c = 0; c < DIM; ++c) r[c] = pi[c] - src[c * ns + s];
                        const double r2 = DIM == 3 ? dist2(r[0], r[1], r[2]) : dist2(r[0], r[1]);
                        if (r2 < sc.cut2) fn(pass == 1, s, r, r2);
                    }
                }
            }
        }
    }
}

template <int DIM>
void HostExec::density(bool use_dt)
{
    const int64_t n = N_;
    const auto chunks = host_chunks(fo_);
    parallel_chunks((int64_t)chunks.size(), nthreads_, [&](int64_t ci) {
        const HostChunk &hc = chunks[ci];
        const InstDev &I = inst_[hc.b];
        const double dtb = use_dt ? buf_.dt[hc.b] : 0.0;
        for (int64_t k = hc.begin; k < hc.end; ++k) {
            double pi[3] = {0, 0, 0}, vi[3] = {0, 0, 0};
            for (int c = 0; c < DIM; ++c) {
                pi[c] = xs_[c * n + k];
                vi[c] = vs_[c * n + k];
            }
            double sigma = sc_.W0, drho = 0.0;
            int cnt = 0;
            host_neighbours<DIM>(sc_, I, skey_[k] - I.cell_base, k, pi, buf_.cell_start, buf_.wall_start,
                                 xs_.data(), n, xws_.data(), Nw_,
                                 [&](bool wall, int s, const double *r, double r2) {
                                     double vj[3] = {0, 0, 0};
                                     if (!wall)
                                         for (int c = 0; c < DIM; ++c) vj[c] = vs_[c * n + s];
                                     density_pair<DIM, double>(r, r2, vi, vj, sc_.inv_h, sc_.kW, sc_.kF, sigma,
                                                               drho, cnt);
                                 });
            const int i = buf_.perm[k];
            double rn, P;
            density_update(buf_.rho[i], sigma, sc_.mass * drho, dtb, sc_.mass, sc_.rho0, I.c0, rn, P);
            buf_.rho[i] = rn;
            buf_.count[i] = cnt;
            rhos_[k] = rn;
            Ps_[k] = P;
        }
    });
}

template <int DIM>
void HostExec::force(bool fused)
{
    const int64_t n = N_;
    const auto chunks = host_chunks(fo_);
    vals_.assign(chunks.size() * kNPart, 0.0);
    parallel_chunks((int64_t)chunks.size(), nthreads_, [&](int64_t ci) {
        const HostChunk &hc = chunks[ci];
        const InstDev &I = inst_[hc.b];
        const double dtb = fused ? buf_.dt[hc.b] : 0.0;
        double *tot = vals_.data() + ci * kNPart;
        for (int64_t k = hc.begin; k < hc.end; ++k) {
            double pi[3] = {0, 0, 0}, vi[3] = {0, 0, 0};
            for (int c = 0; c < DIM; ++c) {
                pi[c] = xs_[c * n + k];
                vi[c] = vs_[c * n + k];
            }
            const double rho_i = rhos_[k], P_i = Ps_[k];
            const double p_i = P_i * rho_i * rho_i, inv_rho_i2 = 1.0 / (rho_i * rho_i);
            const double visc_a = sc_.alpha * I.c0 * sc_.h;
            double acc[3] = {0, 0, 0}, aff[3] = {0, 0, 0};
            int cnt = 0;
            host_neighbours<DIM>(sc_, I, skey_[k] - I.cell_base, k, pi, buf_.cell_start, buf_.wall_start,
                                 xs_.data(), n, xws_.data(), Nw_,
                                 [&](bool wall, int s, const double *r, double r2) {
                                     double vj[3] = {0, 0, 0};
                                     double rho_j = 0.0, P_j = 0.0;
                                     if (!wall) {
                                         for (int c = 0; c < DIM; ++c) vj[c] = vs_[c * n + s];
                                         rho_j = rhos_[s];
                                         P_j = Ps_[s];
                                     }
                                     force_pair<DIM, double>(wall, r, r2, vi, vj, rho_i, P_i, p_i, inv_rho_i2, rho_j,
                                                             P_j, sc_.inv_h, sc_.kF, visc_a, sc_.eps_h2, sc_.g[0],
                                                             sc_.g[1], sc_.g[2], acc, aff, cnt);
                                 });
            const int i = buf_.perm[k];
            double vals[kNPart];
            for (int q = 0; q < kNPart; ++q) vals[q] = 0.0;
            double an[DIM], vn[DIM], xi[DIM];
            for (int c = 0; c < DIM; ++c) {
                an[c] = sc_.g[c] + sc_.mass * acc[c];
                buf_.a[c * n + i] = an[c];
                vals[P_FF + c] = sc_.mass * (sc_.mass * aff[c]);
                vn[c] = buf_.v[c * n + i];
                if (fused) {
                    vn[c] = kick(vn[c], an[c], dtb);
                    buf_.v[c * n + i] = vn[c];
                }
                xi[c] = buf_.x[c * n + i];
            }
            vals[P_PAIRS] = (double)cnt;
            state_partials<DIM>(sc_, I, vn, an, xi, buf_.rho[i], vals);
            for (int q = 0; q < kNPart; ++q) tot[q] = is_max_slot(q) ? std::max(tot[q], vals[q]) : tot[q] + vals[q];
        }
    });
}

// Per instance: the chunks' sums in chunk order, the diagnostics and dt.
void HostExec::reduce(bool prime)
{
    const auto chunks = host_chunks(fo_);
    std::vector<double> tot(inst_.size() * kNPart, 0.0);
    for (size_t ci = 0; ci < chunks.size(); ++ci) {
        double *t = tot.data() + (size_t)chunks[ci].b * kNPart;
        const double *c = vals_.data() + ci * kNPart;
        for (int q = 0; q < kNPart; ++q) t[q] = is_max_slot(q) ? std::max(t[q], c[q]) : t[q] + c[q];
    }
    for (size_t b = 0; b < inst_.size(); ++b) {
        const InstDev &I = inst_[b];
        const double *t = tot.data() + b * kNPart;
        double *d = buf_.diag + b * SPH_NDIAG;
        const double dt_used = prime ? 0.0 : buf_.dt[b];
        fill_diag(sc_, I, t, dt_used, clamped_[b], prime ? 1 : 0, d);
        clamped_[b] = 0;
        buf_.dt[b] = cfl_dt(sc_, I.c0, t[P_VMAX], t[P_AMAX]);
        if (t[P_BAD] > 0.0) flags_ |= SPH_FLAG_NONFINITE;
    }
}

void HostExec::prime()
{
    std::fill(buf_.diag, buf_.diag + inst_.size() * SPH_NDIAG, 0.0);
    std::fill(clamped_.begin(), clamped_.end(), 0);
    if (sc_.dim == 2) {
        keys<2>(false);
        sort(false);
        pack<2>();
        density<2>(false);
        force<2>(false);
    } else {
        keys<3>(false);
        sort(false);
        pack<3>();
        density<3>(false);
        force<3>(false);
    }
    reduce(true);
    steps_ = 0;
}

void HostExec::step()
{
    const bool ro = K_ > 0 && (steps_ % K_) == 0;
    if (sc_.dim == 2) {
        keys<2>(true);
        sort(ro);
        pack<2>();
        density<2>(true);
        force<2>(true);
    } else {
        keys<3>(true);
        sort(ro);
        pack<3>();
        density<3>(true);
        force<3>(true);
    }
    reduce(false);
    ++steps_;
}

}  // namespace sphx
