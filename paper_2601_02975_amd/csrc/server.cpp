// Solve server: continuous admission of solve requests into a fixed number
// of slots on one device.  Each slot is a host thread with its own
// non-blocking HIP stream; a request runs mg_solve on its problem's resident
// hierarchy, so the solves of different requests overlap on the device and a
// request's result is the one mg_solve gives alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mg.h"

namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0, Clock::time_point t) {
    return std::chrono::duration<double>(t - t0).count();
}

struct Problem {
    mg_grid grid{};
    std::vector<std::vector<mg_segment>> segs;
    double a = 0, b = 0, c = 0;
    mg_options opt{};
    mg_handle h = nullptr;
    long long bytes = 0;          // device bytes of the hierarchy (estimate until set up)
    double sweep_bytes = 0;       // smoother SFV bytes of one outer iteration (once set up)
    bool busy = false, failed = false;
    mg_status setup_status = MG_OK;
    std::string setup_error;
    long long last_used = 0;
};

struct Request {
    int problem = 0;
    const double *f = nullptr, *g = nullptr;
    double *u = nullptr;
    double tol = 0;
    Clock::time_point t_submit, t_start, t_done;
    bool done = false;
    mg_status status = MG_OK;
    int iters = 0;
    double rel = 0;
    std::string error;            // mg_last_error() of a failed setup or solve
};

// device bytes a hierarchy is assumed to need before its setup has run:
// about 80 bytes per finest-level cell over all levels, plus a dense bottom
// inverse of up to 64 MiB
long long footprint_estimate(const mg_grid &g) { return 80LL * g.nx * g.ny + (64LL << 20); }

}  // namespace

struct mg_server_s {
    mg_server_options opt{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Problem> problems;                  // stable references while slots run
    std::map<unsigned long long, Request> reqs;
    std::deque<unsigned long long> queue;
    unsigned long long next_ticket = 1;
    long long resident_bytes = 0, tick = 0;
    int active = 0, evictions = 0;
    long long submitted = 0, completed = 0, failed = 0;
    double moved_bytes = 0;                        // smoother SFV bytes of the completed solves
    bool stopping = false, any_submit = false;
    Clock::time_point t_first_submit, t_last_done;
    std::vector<double> latencies, solve_times;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;

    // A request that can start now: its problem is idle and either resident
    // or admissible, possibly after evicting idle resident hierarchies (least
    // recently used first).  Admission is decided before anything is
    // evicted: hierarchies are evicted only when that makes the request fit
    // (or when nothing else would stay resident, so that a request larger
    // than the budget still runs alone).  The evicted handles are returned
    // in `victims`, to be destroyed after mu is released.  Called with mu
    // held.
    bool pick(unsigned long long &ticket, std::vector<mg_handle> &victims) {
        for (auto it = queue.begin(); it != queue.end(); ++it) {
            Request &r = reqs[*it];
            Problem &p = problems[r.problem];
            if (p.busy) continue;
            if (!p.h && !p.failed) {
                const long long need = footprint_estimate(p.grid);
                long long idle = 0;
                for (const Problem &q : problems)
                    if (q.h && !q.busy) idle += q.bytes;
                const long long busy_bytes = resident_bytes - idle;
                const bool fits_after_eviction = busy_bytes + need <= opt.hbm_budget;
                const bool runs_alone = busy_bytes == 0;
                if (!fits_after_eviction && !runs_alone) continue;
                while (resident_bytes + need > opt.hbm_budget) {
                    int victim = -1;
                    for (int k = 0; k < (int)problems.size(); ++k) {
                        const Problem &q = problems[k];
                        if (q.h && !q.busy && (victim < 0 || q.last_used < problems[victim].last_used)) victim = k;
                    }
                    if (victim < 0) break;
                    victims.push_back(problems[victim].h);
                    problems[victim].h = nullptr;
                    resident_bytes -= problems[victim].bytes;
                    problems[victim].bytes = 0;
                    ++evictions;
                }
                resident_bytes += need;
                p.bytes = need;
            }
            ticket = *it;
            queue.erase(it);
            return true;
        }
        return false;
    }

    void worker(int slot) {
        (void)hipSetDevice(device);
        hipStream_t st = streams[slot];
        std::unique_lock<std::mutex> lk(mu);
        while (true) {
            unsigned long long ticket = 0;
            std::vector<mg_handle> victims;
            cv_work.wait(lk, [&] { return stopping || pick(ticket, victims); });
            if (!ticket) return;                       // stopping with nothing to start
            Request &r = reqs[ticket];
            Problem &p = problems[r.problem];
            p.busy = true;
            p.last_used = ++tick;
            ++active;
            r.t_start = Clock::now();
            lk.unlock();
            for (mg_handle v : victims) mg_destroy(v);
            mg_status rc = MG_OK;
            std::string err;
            if (p.failed) {
                rc = p.setup_status;
                err = p.setup_error;
            } else if (!p.h) {
                std::vector<mg_curve> cv(p.segs.size());
                for (size_t k = 0; k < p.segs.size(); ++k) cv[k] = {(int)p.segs[k].size(), p.segs[k].data()};
                mg_handle h = nullptr;
                rc = mg_setup(&p.grid, (int)cv.size(), cv.data(), p.a, p.b, p.c, &p.opt, st, &h);
                mg_info info{};
                if (rc == MG_OK) mg_query(h, &info);
                else err = mg_last_error();
                lk.lock();
                resident_bytes -= p.bytes;
                if (rc == MG_OK) {
                    p.h = h;
                    p.bytes = info.device_bytes;
                    resident_bytes += p.bytes;
                    // one V-cycle: nu1 + nu2 sweeps on every level above the
                    // bottom, each reading u and b and writing u on the SFV cells
                    const double w = p.opt.precision == MG_MIXED ? 4.0 : 8.0;
                    p.sweep_bytes = 0;
                    for (int l = 0; l + 1 < info.n_levels && l < 16; ++l)
                        p.sweep_bytes += (p.opt.nu1 + p.opt.nu2) * 3.0 * w * (double)info.n_sfv[l];
                } else {
                    p.failed = true;
                    p.setup_status = rc;
                    p.setup_error = err;
                    p.bytes = 0;
                }
                lk.unlock();
            }
            int iters = 0;
            double rel = 0;
            if (rc == MG_OK) {
                rc = mg_solve(p.h, r.f, r.g, r.u, r.tol, st, &iters, &rel);
                if (rc != MG_OK) err = mg_last_error();
            }
            const auto t = Clock::now();
            lk.lock();
            r.status = rc;
            r.error = err;
            r.iters = iters;
            r.rel = rel;
            r.t_done = t;
            r.done = true;
            p.busy = false;
            p.last_used = ++tick;
            --active;
            if (rc == MG_OK) {
                ++completed;
                moved_bytes += iters * p.sweep_bytes;
                latencies.push_back(seconds_since(r.t_submit, t));
                solve_times.push_back(seconds_since(r.t_start, t));
                t_last_done = t;
            } else {
                ++failed;
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }
};

namespace {

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const size_t k = (size_t)std::min<double>((double)v.size() - 1, std::ceil(q * v.size()) - 1);
    return v[k];
}

}  // namespace

extern "C" {

mg_status mg_server_create(const mg_server_options *opt, mg_server *out) {
    if (!opt || !out || opt->max_active < 1 || opt->max_active > 64 || opt->hbm_budget <= 0) return MG_ERR_INVALID_ARG;
    *out = nullptr;
    auto s = new mg_server_s();
    s->opt = *opt;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return MG_ERR_HIP;
    }
    s->streams.resize(opt->max_active, nullptr);
    for (auto &st : s->streams)
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto &x : s->streams)
                if (x) (void)hipStreamDestroy(x);
            delete s;
            return MG_ERR_HIP;
        }
    for (int k = 0; k < opt->max_active; ++k) s->workers.emplace_back([s, k] { s->worker(k); });
    *out = s;
    return MG_OK;
}

mg_status mg_server_add_problem(mg_server s, const mg_grid *grid, int n_curves, const mg_curve *curves, double a,
                                double b, double c, const mg_options *opt, int *problem) {
    if (!s || !grid || !curves || n_curves < 1 || !problem) return MG_ERR_INVALID_ARG;
    Problem p;
    p.grid = *grid;
    for (int k = 0; k < n_curves; ++k) {
        if (curves[k].n_seg < 1 || !curves[k].seg) return MG_ERR_INVALID_ARG;
        p.segs.emplace_back(curves[k].seg, curves[k].seg + curves[k].n_seg);
    }
    p.a = a; p.b = b; p.c = c;
    mg_default_options(&p.opt);
    if (opt) p.opt = *opt;
    std::lock_guard<std::mutex> lk(s->mu);
    s->problems.push_back(std::move(p));
    *problem = (int)s->problems.size() - 1;
    return MG_OK;
}

mg_status mg_server_submit(mg_server s, int problem, const double *f_dev, const double *g_dev, double *u_dev,
                           double tol, unsigned long long *ticket) {
    if (!s || !f_dev || !u_dev || !(tol > 0) || !ticket) return MG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (problem < 0 || problem >= (int)s->problems.size() || s->stopping) return MG_ERR_INVALID_ARG;
    Request r;
    r.problem = problem;
    r.f = f_dev;
    r.g = g_dev;
    r.u = u_dev;
    r.tol = tol;
    r.t_submit = Clock::now();
    if (!s->any_submit) {
        s->any_submit = true;
        s->t_first_submit = r.t_submit;
    }
    const unsigned long long t = s->next_ticket++;
    s->reqs[t] = r;
    s->queue.push_back(t);
    ++s->submitted;
    *ticket = t;
    s->cv_work.notify_one();
    return MG_OK;
}

mg_status mg_server_poll(mg_server s, unsigned long long ticket, int *done, mg_status *status, int *iters,
                         double *rel_residual, double *latency_s) {
    if (!s) return MG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return MG_ERR_INVALID_ARG;
    const Request &r = it->second;
    if (done) *done = r.done ? 1 : 0;
    if (r.done) {
        if (status) *status = r.status;
        if (iters) *iters = r.iters;
        if (rel_residual) *rel_residual = r.rel;
        if (latency_s) *latency_s = seconds_since(r.t_submit, r.t_done);
    }
    return MG_OK;
}

mg_status mg_server_wait(mg_server s, unsigned long long ticket, mg_status *status, int *iters, double *rel_residual,
                         double *latency_s) {
    if (!s) return MG_ERR_INVALID_ARG;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return MG_ERR_INVALID_ARG;
        s->cv_done.wait(lk, [&] { return it->second.done; });
    }
    return mg_server_poll(s, ticket, nullptr, status, iters, rel_residual, latency_s);
}

const char *mg_server_request_error(mg_server s, unsigned long long ticket) {
    if (!s) return "";
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    return it == s->reqs.end() ? "" : it->second.error.c_str();
}

mg_status mg_server_get_stats(mg_server s, mg_server_stats *st) {
    if (!s || !st) return MG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *st = mg_server_stats{};
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->failed = s->failed;
    st->p50_latency_s = percentile(s->latencies, 0.50);
    st->p99_latency_s = percentile(s->latencies, 0.99);
    st->p50_solve_s = percentile(s->solve_times, 0.50);
    st->p99_solve_s = percentile(s->solve_times, 0.99);
    if (s->completed > 0) {
        const double span = seconds_since(s->t_first_submit, s->t_last_done);
        st->solves_per_s = span > 0 ? s->completed / span : 0.0;
        st->sweep_gbs = span > 0 ? s->moved_bytes / span / 1e9 : 0.0;
    }
    st->resident_bytes = s->resident_bytes;
    for (const auto &p : s->problems) st->resident_problems += p.h != nullptr;
    st->evictions = s->evictions;
    return MG_OK;
}

mg_status mg_server_destroy(mg_server s) {
    if (!s) return MG_OK;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->queue.empty() && s->active == 0; });
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    for (auto &p : s->problems)
        if (p.h) mg_destroy(p.h);
    for (auto &st : s->streams) (void)hipStreamDestroy(st);
    delete s;
    return MG_OK;
}

}  // extern "C"
