// Serving many independent boxes on one GPU: a first-in first-out queue with
// admission against an HBM budget, and one host thread, HIP stream and
// context per slot so that several boxes run concurrently.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/cube.h"
#include "internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
    cube_request req{};
    int64_t footprint = 0;
    bool done = false;
    cube_result res{};
};

}  // namespace

struct cube_server {
    cube_server_desc d{};
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;                    // waiting tickets, oldest first
    std::unordered_map<uint64_t, Job> jobs;
    int64_t in_use = 0;                            // footprints of the running boxes
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::vector<std::thread> slots;

    double now_ms() const { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }
    void slot_loop();
};

namespace {

cube_status fail(cube_status st, const std::string& msg) {
    cube::set_last_error(msg.c_str());
    return st;
}

void note_error(cube_result& r, cube_status st) {
    r.status = st;
    const char* m = cube_last_error();
    std::strncpy(r.message, m ? m : "", sizeof(r.message) - 1);
    r.message[sizeof(r.message) - 1] = 0;
}

// one box, start to finish, on this thread's own stream and context
void run_box(const cube_server_desc& sd, Job& j) {
    cube_result& r = j.res;
    if (hipSetDevice(sd.device) != hipSuccess) {
        r.status = CUBE_DEVICE;
        std::strncpy(r.message, "hipSetDevice failed", sizeof(r.message) - 1);
        return;
    }
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        r.status = CUBE_DEVICE;
        std::strncpy(r.message, "hipStreamCreate failed", sizeof(r.message) - 1);
        return;
    }
    cube_box_desc desc = j.req.desc;
    if (sd.precision >= 0) desc.precision = sd.precision;
    cube_ctx* c = nullptr;
    cube_status st = cube_init(&desc, nullptr, s, &c);
    if (st == CUBE_OK) st = cube_compress(c, j.req.pos, j.req.vel, j.req.n, 0);
    if (st == CUBE_OK) {
        st = cube_pm_step(c, j.req.n_steps);
        if (st == CUBE_OK) r.steps_done = j.req.n_steps;
    }
    if (st == CUBE_OK && j.req.want_diag) st = cube_diagnostics(c, &r.diag);
    if (st == CUBE_OK && j.req.out_state) st = cube_get_state(c, j.req.out_state);
    if (st != CUBE_OK) note_error(r, st);
    else r.status = CUBE_OK;
    cube_destroy(c);
    hipStreamDestroy(s);
}

}  // namespace

void cube_server::slot_loop() {
    for (;;) {
        uint64_t t = 0;
        Job* j = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            // strict FIFO: only the head may start, so a large box is never overtaken forever
            cv.wait(lk, [&] {
                return stopping || (!queue.empty() && in_use + jobs[queue.front()].footprint <= d.hbm_budget_bytes);
            });
            if (stopping) return;
            t = queue.front();
            queue.pop_front();
            j = &jobs[t];
            in_use += j->footprint;
            j->res.start_ms = now_ms();
            cv.notify_all();            // the next head may fit as well
        }
        run_box(d, *j);
        {
            std::lock_guard<std::mutex> lk(mu);
            in_use -= j->footprint;
            j->res.done_ms = now_ms();
            j->done = true;
        }
        cv.notify_all();
    }
}

extern "C" {

cube_status cube_server_create(const cube_server_desc* desc, cube_server** out) {
    if (!out) return fail(CUBE_INVALID, "null output pointer");
    *out = nullptr;
    if (!desc || desc->max_slots < 1 || desc->hbm_budget_bytes <= 0 || desc->precision < -1 ||
        desc->precision > CUBE_MIXED_FP16)
        return fail(CUBE_INVALID, "server needs max_slots >= 1, a positive budget and a known precision");
    cube_server* srv = new cube_server();
    srv->d = *desc;
    srv->t0 = Clock::now();
    for (int i = 0; i < desc->max_slots; ++i) srv->slots.emplace_back([srv] { srv->slot_loop(); });
    *out = srv;
    return CUBE_OK;
}

cube_status cube_submit(cube_server* srv, const cube_request* req, uint64_t* ticket) {
    if (!srv || !req || !ticket) return fail(CUBE_INVALID, "null argument");
    if (!req->pos || !req->vel || req->n_steps < 0) return fail(CUBE_INVALID, "request needs pos, vel and n_steps >= 0");
    cube_box_desc desc = req->desc;
    if (srv->d.precision >= 0) desc.precision = srv->d.precision;
    int64_t pers = 0, trans = 0;
    cube_status st = cube_footprint(&desc, &pers, &trans);
    if (st != CUBE_OK) return st;    // cube_footprint set the message
    const int64_t n = (int64_t)desc.n_side * desc.n_side * desc.n_side;
    if (req->n != n) return fail(CUBE_INVALID, "request needs n_side^3 particles");
    const int64_t need = pers + trans;
    if (need > srv->d.hbm_budget_bytes)
        return fail(CUBE_INVALID, "box needs " + std::to_string(need) + " device bytes, above the whole budget");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stopping) return fail(CUBE_INVALID, "server is shutting down");
        const uint64_t t = srv->next_ticket++;
        Job& j = srv->jobs[t];
        j.req = *req;
        j.footprint = need;
        j.res.footprint_bytes = need;
        j.res.submit_ms = srv->now_ms();
        j.res.status = CUBE_NOT_READY;
        srv->queue.push_back(t);
        *ticket = t;
    }
    srv->cv.notify_all();
    return CUBE_OK;
}

cube_status cube_poll(cube_server* srv, uint64_t ticket, cube_result* out) {
    if (!srv || !out) return fail(CUBE_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end()) return fail(CUBE_INVALID, "unknown ticket");
    if (!it->second.done) return CUBE_NOT_READY;
    *out = it->second.res;
    srv->jobs.erase(it);
    return CUBE_OK;
}

void cube_server_destroy(cube_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
    }
    srv->cv.notify_all();
    for (std::thread& t : srv->slots) t.join();
    delete srv;
}

}  // extern "C"
