// Serving engine: map-making solves of several recurring scan strategies,
// continuously batched on one GPU.
//
// Each strategy owns a context (its own HIP stream), its pointing, noise and
// M_BD built at registration, and up to two PCG sessions ("lanes") of `slots`
// lockstep columns: one preconditioned by M_BD, one by M_2l.  M_2l is built
// from the first request's right-hand side and reused for every later request
// of that strategy -- the paper's point that M_2l pays off when the same
// system is solved many times (Sect. 7.3).  The build (Arnoldi, Ritz
// vectors, AZ, E) runs on a host thread of its own with a context and stream
// of its own, so it never holds up other requests: the request that triggers
// it and those admitted before it is ready are solved with M_BD, later ones
// with M_2l.  A step admits queued requests into free slots (computing their b
// on the strategy's stream), runs a chunk of iterations on every lane with
// running slots -- enqueued on all streams before any is waited on, so
// strategies overlap on the device -- and retires finished slots, writing
// each solution to the caller's buffer.
//
// Memory is admitted against a byte budget in two parts.  A strategy's
// resident data (pointing, noise, M_BD, the M_2l build's reserve) is charged
// when it is registered.  A lane's session -- its `slots` columns of PCG
// vectors and the strategy context's TOD workspaces for that many columns --
// is charged when the lane first admits a request, and stays (cached) while
// memory allows; a request whose lane has no session and whose session does
// not fit waits for memory, and idle sessions of other lanes are evicted (their
// memory freed) to make room.  A request joining a session with a free slot
// needs no new memory; one whose session is full waits for a slot.
#include <atomic>
#include <chrono>
#include <deque>
#include <map>
#include <memory>
#include <thread>

#include "mm_internal.h"

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    int64_t id = 0;
    int32_t strategy = 0;
    const void *tod = nullptr;
    double *x_out = nullptr;
    double tol = 1e-8;
    int32_t max_iter = 1000;
    int32_t state = 0;  // 0 queued, 1 running, 2 converged, 3 budget spent, 4 failed
    int32_t slot = -1;
    int32_t iters = 0;
    double rel_res = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
    int32_t m2l_built = 0;  // 1 if this request triggered the M_2l build
    int32_t lane = 0;       // 0 = M_BD session, 1 = M_2l session
    int32_t waited = 0;     // what it waited for before admission: 1 slot, 2 memory
};

// One PCG session of a strategy and the request held by each of its slots.
struct Lane {
    mm_pcg *sess = nullptr;
    int64_t charged = 0;  // bytes of the budget this session holds
    std::vector<int64_t> slot_req;
    bool busy() const {
        for (auto q : slot_req)
            if (q >= 0) return true;
        return false;
    }
};

enum BuildState { BUILD_NONE = 0, BUILD_RUNNING = 1, BUILD_READY = 2, BUILD_FAILED = 3 };

struct Strategy {
    int32_t id = 0;
    mm_ctx *ctx = nullptr;
    mm_pointing *p = nullptr;
    mm_noise *nz = nullptr;
    mm_precond *mbd = nullptr;
    mm_precond *m2l = nullptr;  // adopted once the background build is ready
    Lane lane[2];
    mm::DBuf b;
    int64_t bytes = 0;         // resident part, charged at registration
    int64_t session_bytes = 0; // one lane session of `slots` columns
    int64_t n = 0;
    // background M_2l build: its own context and stream, seeded with a copy
    // of the first request's b; it only reads p, nz and mbd
    std::thread builder;
    std::atomic<int> build{BUILD_NONE};
    mm_ctx *bctx = nullptr;
    mm_precond *m2l_new = nullptr;
    mm::DBuf b_seed;
    void join_builder() {
        if (builder.joinable()) builder.join();
        mm_ctx_destroy(bctx);
        bctx = nullptr;
    }
    ~Strategy() {
        join_builder();
        mm_precond_destroy(m2l_new);
        for (auto &l : lane) mm_pcg_destroy(l.sess);
        mm_precond_destroy(m2l);
        mm_precond_destroy(mbd);
        mm_noise_destroy(nz);
        mm_pointing_destroy(p);
        b.release();
        b_seed.release();
        mm_ctx_destroy(ctx);
    }
};

}  // namespace

struct mm_server {
    int device = 0;
    int64_t budget = 0;
    int64_t used = 0;
    int32_t slots = 8;
    int32_t defl_k = 32;
    int32_t chunk = 4;
    int32_t m_max = 256;
    double eps_arn = 1e-8;
    int32_t arn_stop = MM_ARN_STOP_H;  // stop rule of the background Arnoldi
    // build M_2l at registration (synchronously, on the strategy's stream)
    // from the Ritz vectors of an M_BD solve of A x = A u, u a fixed
    // pseudo-random map, instead of in the background from the first request
    bool prebuild = false;
    int64_t next_id = 1;
    std::map<int32_t, std::unique_ptr<Strategy>> strat;
    std::deque<int64_t> queue;
    std::map<int64_t, Request> req;
    std::string last_error;
};

using namespace mm;

#define SRV_TRY try {
#define SRV_END                                               \
    }                                                         \
    catch (const mm::Error &e) {                              \
        srv->last_error = e.what();                           \
        return e.code;                                        \
    }                                                         \
    catch (const std::exception &e) {                         \
        srv->last_error = e.what();                           \
        return MM_E_DEVICE;                                   \
    }

static void check(mm_status st, mm_ctx *ctx, const char *what) {
    if (st < 0) throw Error(st, std::string(what) + ": " + mm_last_error(ctx));
}

// Resident footprint of a strategy: per sample, the pointing (compact pixel,
// weights, permutation, sorted weights, the angle in the FP64 form, the
// sliced P^T entries with ~10 % padding, P's map-copy slot with a grid);
// per unknown, M_BD (its inverse blocks and its assembled blocks), b and the
// M_2l reserve (Z, AZ, the Arnoldi basis); and the single-column TOD
// workspaces of the M_2l builder's context.
static int64_t resident_bytes(const mm_server *srv, int64_t n_samp, int64_t est_n, int64_t te,
                              bool grid) {
    const int64_t per_samp = 4 + 2 * 2 * te + 4 + (te == 4 ? 0 : 8) + 14 + (grid ? 4 : 0);
    return n_samp * per_samp + 2 * n_samp * te +
           est_n * 8 * (6 + 2 * srv->defl_k + srv->m_max + 2);
}

// One lane session of `slots` columns: the session's column vectors (x, r,
// z, p, q) and its single-column buffer, its two sets of per-block partial
// sums (at most 512 blocks per column), the strategy context's TOD
// workspaces for `slots` columns, and the sliced P^T's partial maps of the
// right-hand side.
static int64_t session_bytes(const mm_server *srv, int64_t n_samp, int64_t n, int64_t n_obs,
                             int64_t te) {
    return 8 * n * (5 * (int64_t)srv->slots + 1) + 2 * 8 * 512 * (int64_t)srv->slots +
           2 * n_samp * te * srv->slots + 8 * 3 * n_obs * 64;
}

extern "C" mm_status mm_server_create(int device, int64_t hbm_budget_bytes, int32_t slots,
                                      int32_t defl_k, int32_t iters_per_step,
                                      mm_server **out) {
    if (!out) return MM_E_INVALID;
    *out = nullptr;
    if (hbm_budget_bytes <= 0 || !pow2_ok(slots) || defl_k < 0 || defl_k > 63 ||
        iters_per_step < 1)
        return MM_E_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return MM_E_INVALID;
    auto *s = new mm_server();
    s->device = device;
    s->budget = hbm_budget_bytes;
    s->slots = slots;
    s->defl_k = defl_k;
    s->chunk = iters_per_step;
    *out = s;
    return MM_OK;
}

extern "C" mm_status mm_server_set_prebuild(mm_server *srv, int32_t on) {
    if (!srv) return MM_E_INVALID;
    srv->prebuild = on != 0;
    return MM_OK;
}

extern "C" mm_status mm_server_set_arnoldi(mm_server *srv, int32_t stop_rule, double eps_arn,
                                           int32_t m_max) {
    if (!srv) return MM_E_INVALID;
    if (stop_rule != MM_ARN_STOP_H && stop_rule != MM_ARN_STOP_RESIDUAL) return MM_E_INVALID;
    if (!(eps_arn >= 0) || m_max < 1 || m_max > 500) return MM_E_INVALID;
    if (!srv->strat.empty()) {
        srv->last_error = "server: the Arnoldi parameters are set before any strategy";
        return MM_E_INVALID;
    }
    srv->arn_stop = stop_rule;
    srv->eps_arn = eps_arn;
    srv->m_max = m_max;
    return MM_OK;
}

extern "C" const char *mm_server_last_error(const mm_server *srv) {
    return srv ? srv->last_error.c_str() : "null server";
}

extern "C" mm_status mm_server_add_strategy(mm_server *srv, int32_t id, int64_t n_samp,
                                            int32_t n_pix_total, const int32_t *pix,
                                            const double *psi, int32_t min_hits,
                                            int32_t grid_width, int32_t n_intervals,
                                            const int64_t *interval_start,
                                            const int32_t *filter_id, int32_t n_filters,
                                            int32_t half_bw, const double *band,
                                            mm_precision prec) {
    if (!srv) return MM_E_INVALID;
    SRV_TRY
    MM_CHECK(!srv->strat.count(id), MM_E_INVALID, "server: strategy id already registered");
    MM_CHECK(n_samp > 0 && n_pix_total > 0 && n_intervals > 0, MM_E_INVALID,
             "server: bad strategy sizes");
    // footprint: pointing (index, weights, permutation, sorted weights; the
    // FP64 form also keeps the angles; with a grid, P's map-copy slot per
    // sample), the sliced P^T layout (index and angle or weights per entry,
    // ~10 % padding), two TOD workspaces of
    // `slots` columns plus the single-column ones of the M_2l build, two
    // sessions' vectors, M_2l (Z, AZ, W basis)
    const int64_t te = prec == MM_F32 ? 4 : 8;
    const int64_t est_n = 3 * (int64_t)std::min<int64_t>(n_pix_total, n_samp);
    const int64_t bytes = resident_bytes(srv, n_samp, est_n, te, grid_width > 0);
    // its resident part, and room for one lane session once the other
    // strategies' sessions are evicted
    const int64_t sess = session_bytes(srv, n_samp, est_n, est_n / 3, te);
    if (srv->used + bytes + sess > srv->budget)
        throw Error(MM_E_BUSY, "server: strategy footprint " + std::to_string(bytes) + " B + " +
                                   std::to_string(sess) +
                                   " B for a session exceeds the remaining budget");
    auto st = std::make_unique<Strategy>();
    st->id = id;
    check(mm_ctx_create(srv->device, nullptr, &st->ctx), nullptr, "server: context");
    check(mm_pointing_build(st->ctx, n_samp, n_pix_total, pix, psi, min_hits, prec, &st->p),
          st->ctx, "server: pointing");
    if (grid_width > 0) check(mm_pointing_set_grid(st->ctx, st->p, grid_width), st->ctx, "grid");
    check(mm_noise_build(st->ctx, n_intervals, interval_start, filter_id, n_filters, half_bw, band,
                         MM_NOISE_AUTO, prec, &st->nz),
          st->ctx, "server: noise");
    check(mm_mbd_build(st->ctx, st->p, st->nz, &st->mbd), st->ctx, "server: M_BD");
    st->n = st->p->n();
    st->b.alloc(sizeof(double) * st->n);
    if (srv->prebuild && srv->defl_k > 0) {
        // b = A u for a fixed u with entries uniform in [-1, 1): a consistent
        // right-hand side whose Krylov space holds every eigenvector of M_BD A
        std::vector<double> hu((size_t)st->n);
        uint64_t z = 0x9E3779B97F4A7C15ull ^ (uint64_t)id;
        for (auto &v : hu) {  // splitmix64
            z += 0x9E3779B97F4A7C15ull;
            uint64_t q = z;
            q = (q ^ (q >> 30)) * 0xBF58476D1CE4E5B9ull;
            q = (q ^ (q >> 27)) * 0x94D049BB133111EBull;
            q ^= q >> 31;
            v = 2.0 * (double)(q >> 11) * 0x1.0p-53 - 1.0;
        }
        mm::DBuf u;
        u.alloc(sizeof(double) * st->n);
        MM_HIP(hipMemcpyAsync(u.ptr, hu.data(), sizeof(double) * st->n, hipMemcpyHostToDevice,
                              st->ctx->stream));
        check(mm_apply_A(st->ctx, st->p, st->nz, 1, u.as<double>(), st->b.as<double>()),
              st->ctx, "server: prebuild A u");
        const int k = (int)std::min<int64_t>(srv->defl_k, st->n - 1);
        const int mmax = (int)std::min<int64_t>(srv->m_max, st->n);
        check(mm_defl_build_pcg(st->ctx, st->p, st->nz, st->mbd, st->b.as<double>(), k, 0.0,
                                1e-12, mmax, nullptr, nullptr, nullptr, &st->m2l),
              st->ctx, "server: prebuild M_2l");
        st->build = BUILD_READY;
    }
    for (auto &l : st->lane) l.slot_req.assign(srv->slots, -1);
    st->bytes = bytes;
    st->session_bytes = session_bytes(srv, n_samp, st->n, st->p->n_obs, te);
    srv->used += bytes;
    srv->strat[id] = std::move(st);
    SRV_END
    return MM_OK;
}

extern "C" mm_status mm_server_submit(mm_server *srv, int32_t strategy, const void *tod,
                                      double tol, int32_t max_iter, double *x_out,
                                      int64_t *request_id) {
    if (!srv) return MM_E_INVALID;
    SRV_TRY
    MM_CHECK(srv->strat.count(strategy), MM_E_INVALID, "server: unknown strategy");
    MM_CHECK(tod && x_out && tol >= 0 && max_iter >= 1, MM_E_INVALID, "server: bad request");
    Request r;
    r.id = srv->next_id++;
    r.strategy = strategy;
    r.tod = tod;
    r.x_out = x_out;
    r.tol = tol;
    r.max_iter = max_iter;
    r.t_submit = now_s();
    srv->req[r.id] = r;
    srv->queue.push_back(r.id);
    if (request_id) *request_id = r.id;
    SRV_END
    return MM_OK;
}

// Adopt a finished background build (the M_2l lane takes requests admitted
// from now on).
static void poll_build(Strategy &st) {
    const int b = st.build.load();
    if (b == BUILD_READY && !st.m2l) {
        st.join_builder();
        st.m2l = st.m2l_new;
        st.m2l_new = nullptr;
    } else if (b == BUILD_FAILED && st.builder.joinable()) {
        st.join_builder();
    }
}

static void start_build(mm_server *srv, Strategy &st) {
    st.b_seed.alloc(sizeof(double) * st.n);
    MM_HIP(hipMemcpyAsync(st.b_seed.ptr, st.b.ptr, sizeof(double) * st.n,
                          hipMemcpyDeviceToDevice, st.ctx->stream));
    MM_HIP(hipStreamSynchronize(st.ctx->stream));
    const int k = (int)std::min<int64_t>(srv->defl_k, st.n - 1);
    const int mmax = (int)std::min<int64_t>(srv->m_max, st.n);
    const double eps = srv->eps_arn;
    const int32_t rule = srv->arn_stop;
    const int dev = srv->device;
    st.build = BUILD_RUNNING;
    Strategy *sp = &st;
    st.builder = std::thread([sp, k, mmax, eps, rule, dev]() {
        mm_status s = MM_E_DEVICE;
        if (hipSetDevice(dev) == hipSuccess && mm_ctx_create(dev, nullptr, &sp->bctx) == MM_OK)
            s = mm_defl_build_stop(sp->bctx, sp->p, sp->nz, sp->mbd, sp->b_seed.as<double>(), k,
                                   0.0, eps, rule, mmax, nullptr, nullptr, nullptr, &sp->m2l_new);
        sp->build = s >= 0 ? BUILD_READY : BUILD_FAILED;
    });
}

// Free a lane's session and its charge.  With both lanes of the strategy
// idle, the context's TOD workspaces go too.
static void evict(mm_server *srv, Strategy &st, Lane &ln) {
    mm_pcg_destroy(ln.sess);
    ln.sess = nullptr;
    srv->used -= ln.charged;
    ln.charged = 0;
    if (!st.lane[0].sess && !st.lane[1].sess) {
        MM_HIP(hipStreamSynchronize(st.ctx->stream));
        for (mm::DBuf *d : {&st.ctx->tod_a, &st.ctx->tod_b, &st.ctx->tod_c, &st.ctx->pt_part,
                            &st.ctx->xpack})
            d->release();
        ++st.ctx->ws_gen;
    }
}

// Make room for `need` bytes by evicting idle sessions other than `keep`;
// true if the budget then has room.
static bool make_room(mm_server *srv, int64_t need, const Lane *keep) {
    if (srv->used + need <= srv->budget) return true;
    for (auto &kv : srv->strat)
        for (auto &ln : kv.second->lane) {
            if (&ln == keep || !ln.sess || ln.busy()) continue;
            evict(srv, *kv.second, ln);
            if (srv->used + need <= srv->budget) return true;
        }
    return srv->used + need <= srv->budget;
}

// Admit queued requests (FIFO per strategy, no head-of-line blocking across
// strategies) into free slots, creating a lane's session when memory allows.
static void admit(mm_server *srv) {
    for (auto it = srv->queue.begin(); it != srv->queue.end();) {
        Request &r = srv->req[*it];
        Strategy &st = *srv->strat[r.strategy];
        poll_build(st);
        const int li = st.m2l ? 1 : 0;
        Lane &ln = st.lane[li];
        if (!ln.sess && !make_room(srv, st.session_bytes, &ln)) {
            r.waited |= 2;  // waits for memory
            ++it;
            continue;
        }
        int slot = -1;
        for (int c = 0; c < srv->slots; ++c)
            if (ln.slot_req[c] < 0) {
                slot = c;
                break;
            }
        if (slot < 0) {
            r.waited |= 1;  // waits for a slot
            ++it;
            continue;
        }
        mm_ctx *ctx = st.ctx;
        if (!ln.sess) {
            const mm_precond *M = li ? st.m2l : st.mbd;
            check(mm_pcg_create(ctx, st.p, st.nz, M, srv->slots, &ln.sess), ctx, "server: session");
            ln.charged = st.session_bytes;
            srv->used += ln.charged;
        }
        mm_status s = mm_rhs(ctx, st.p, st.nz, 1, r.tod, st.b.as<double>());
        if (s < 0) {
            r.state = 4;
            r.t_done = now_s();
            it = srv->queue.erase(it);
            continue;
        }
        if (!st.m2l && st.build == BUILD_NONE && srv->defl_k > 0) {
            // cache miss: build M_2l from this request's right-hand side, in the background
            start_build(srv, st);
            r.m2l_built = 1;
        }
        check(mm_pcg_start(ctx, ln.sess, slot, st.b.as<double>(), r.tol, r.max_iter), ctx,
              "server: start");
        ln.slot_req[slot] = r.id;
        r.slot = slot;
        r.lane = li;
        r.state = 1;
        r.t_start = now_s();
        it = srv->queue.erase(it);
    }
}

extern "C" mm_status mm_server_step(mm_server *srv, int32_t *n_running, int32_t *n_queued) {
    if (!srv) return MM_E_INVALID;
    SRV_TRY
    admit(srv);
    // enqueue a chunk of iterations on every busy lane, then poll
    for (auto &kv : srv->strat) {
        Strategy &st = *kv.second;
        for (auto &ln : st.lane)
            if (ln.busy()) check(mm_pcg_iterate(st.ctx, ln.sess, srv->chunk), st.ctx, "server: iterate");
    }
    int running = 0;
    std::vector<int32_t> state(srv->slots), iters(srv->slots);
    std::vector<double> rr(srv->slots);
    for (auto &kv : srv->strat) {
        Strategy &st = *kv.second;
        for (auto &ln : st.lane) {
            if (!ln.busy()) continue;
            check(mm_pcg_poll(st.ctx, ln.sess, state.data(), iters.data(), rr.data()), st.ctx,
                  "server: poll");
            for (int c = 0; c < srv->slots; ++c) {
                if (ln.slot_req[c] < 0) continue;
                Request &r = srv->req[ln.slot_req[c]];
                if (state[c] == 1) {
                    ++running;
                    continue;
                }
                r.iters = iters[c];
                r.rel_res = rr[c];
                r.state = state[c] == 2 ? 2 : (state[c] == 3 ? 3 : 4);
                check(mm_pcg_finish(st.ctx, ln.sess, c, r.x_out), st.ctx, "server: finish");
                r.t_done = now_s();
                ln.slot_req[c] = -1;
            }
        }
        poll_build(st);
    }
    if (n_running) *n_running = running;
    if (n_queued) *n_queued = (int32_t)srv->queue.size();
    SRV_END
    return MM_OK;
}

extern "C" mm_status mm_server_strategy_state(mm_server *srv, int32_t strategy,
                                              int32_t *m2l_state) {
    if (!srv || !m2l_state) return MM_E_INVALID;
    SRV_TRY
    auto it = srv->strat.find(strategy);
    MM_CHECK(it != srv->strat.end(), MM_E_INVALID, "server: unknown strategy");
    poll_build(*it->second);
    *m2l_state = it->second->m2l ? BUILD_READY : it->second->build.load();
    SRV_END
    return MM_OK;
}

extern "C" mm_status mm_server_poll(mm_server *srv, int64_t request_id, mm_request_info *info) {
    if (!srv || !info) return MM_E_INVALID;
    SRV_TRY
    auto it = srv->req.find(request_id);
    MM_CHECK(it != srv->req.end(), MM_E_INVALID, "server: unknown request");
    const Request &r = it->second;
    info->state = r.state;
    info->iters = r.iters;
    info->slot = r.slot;
    info->m2l_built = r.m2l_built;
    info->precond = r.state >= 1 ? (r.lane ? 1 : 0) : -1;
    info->waited = r.waited;
    info->rel_res = r.rel_res;
    info->queue_seconds = (r.state >= 1 ? r.t_start : now_s()) - r.t_submit;
    info->latency_seconds = (r.state >= 2 ? r.t_done : now_s()) - r.t_submit;
    SRV_END
    return MM_OK;
}

extern "C" mm_status mm_server_memory(mm_server *srv, int32_t strategy, int64_t *budget,
                                      int64_t *used, int64_t *resident, int64_t *session) {
    if (!srv) return MM_E_INVALID;
    SRV_TRY
    if (budget) *budget = srv->budget;
    if (used) *used = srv->used;
    if (resident || session) {
        auto it = srv->strat.find(strategy);
        MM_CHECK(it != srv->strat.end(), MM_E_INVALID, "server: unknown strategy");
        if (resident) *resident = it->second->bytes;
        if (session) *session = it->second->session_bytes;
    }
    SRV_END
    return MM_OK;
}

extern "C" void mm_server_destroy(mm_server *srv) { delete srv; }
