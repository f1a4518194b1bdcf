// lb_server.cpp -- continuous batching of independent simulations (the
// lb_server_* part of include/lb.h).
//
// A worker thread owns the device side: a compute stream for the batched
// steps and an admission stream (same priority) for setting up new
// simulations.  It loops:
//   1. admit queued requests (FIFO) while the slot count and the device-memory
//      budget allow: create the simulation, upload and initialise its state on
//      the admission stream -- while the chunk launched last (if any) still
//      runs on the compute stream;
//   2. wait for that chunk; drain the simulations it finished (final
//      diagnostics, series copied to the host, apparent viscosity fitted,
//      device memory released, result queued);
//   3. when the set of running simulations changed, rebuild the batch
//      descriptors and the work lists (one entry per CS row or FD tile of
//      every running simulation) and capture one batched step as a HIP graph:
//      one collision-streaming launch, three stage launches per
//      finite-difference equilibrium order, one launch that sums the
//      diagnostics of the simulations sampled in that step, and one that
//      advances the device-side step counter the kernels read;
//   4. launch the next chunk, the step graph replayed once per step; the chunk
//      ends at the first completion (or after chunk_steps).
// Requests that arrive meanwhile wait in the queue and are admitted while the
// next chunk runs, so new work overlaps with running work on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "lb.h"
#include "lb_batch.h"
#include "lb_sim_impl.h"

using namespace lbm;

namespace {

struct Pending {
    uint64_t id;
    lb_request req;
    double t_submit;
    size_t footprint;
    size_t nodes;  // Nx * Ny
    double work;   // estimated device work: nodes x steps x the model's cost per node-step
};

struct Running {
    uint64_t id, tag;
    lb_sim *sim;
    int start_epoch, nsteps, every;
    double t_submit, t_admit;
    size_t footprint, nodes;
    int N;  // FD equilibrium order (0 for CS)
    double dt, decay_k2, decay_omega;  // viscosity fit of the amplitude series (decay_k2 > 0)
};

// Device bytes a request will hold: state buffers, diagnostics partials and
// output, probe vectors and the sample series (as allocated by lb_create,
// lb_set_probe and lb_series_reserve).
size_t footprint_of(const lb_request &r, const ModelInfo &mi)
{
    const bool cs = r.model == LB_CS_D2Q9;
    const size_t nodes = (size_t)r.Nx * r.Ny;
    const size_t plane = (size_t)padded_plane((long long)nodes, (int)sizeof(float));
    // FD buffers hold three FP32 moment planes after the populations
    const size_t state = cs ? 2 * (size_t)mi.K * plane * sizeof(float)
                            : 3 * ((size_t)fd_mom_offset(mi.K, (long long)plane, (int)sizeof(float)) +
                                   3 * plane * sizeof(float));
    int blocks = std::max(cs_diag_blocks(r.Nx, r.Ny), fd_diag_blocks(r.Nx, r.Ny));
    blocks = std::max(blocks, reduce_diag_blocks(r.Nx, r.Ny));
    const size_t diag = sizeof(double) * kDiag * ((size_t)blocks + 1);
    const size_t probe = 2 * (size_t)(r.Nx + r.Ny) * (sizeof(double) + sizeof(float));
    const size_t series = sizeof(double) * kDiag * (size_t)(r.nsteps / r.sample_every + 2);
    return state + diag + probe + series;
}

template <typename T>
struct DevArray {
    T *ptr = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n)
    {
        if (n <= cap) return hipSuccess;
        const size_t want = std::max(n, cap * 2);
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        cap = 0;
        hipError_t e = hipMalloc(&ptr, want * sizeof(T));
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release()
    {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        cap = 0;
    }
};

double now_s(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct lb_server {
    size_t budget = 0;
    int max_slots = 0;
    int chunk = 0;
    int device = 0;
    bool use_graphs = true;  // replay each batched step as a captured graph
    bool tune_tiles = true;  // time the later-stage tile heights per FD order
    // nodes of the simulations admitted at once (0: no limit): enough to
    // fill the device keeps the throughput, and fewer simulations sharing it
    // finish the earlier requests sooner
    size_t node_limit = 0;
    // admission order: arrival (0) or smallest estimated work first (1)
    int policy = 0;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> queue;
    std::deque<lb_result> done;
    std::atomic<bool> stop{false};
    std::atomic<bool> started{false};
    std::thread worker;

    // worker-owned state
    std::vector<Running> running;
    size_t used = 0;
    size_t nodes_in = 0;  // nodes of the admitted simulations
    hipStream_t stream = nullptr;   // batched steps
    hipStream_t astream = nullptr;  // admission: create and initialise new simulations
    hipEvent_t chunk_done = nullptr;
    bool in_flight = false;         // a chunk was launched and not yet waited for
    int epoch = 0;                  // batch steps launched (host mirror of *d_epoch)
    int *d_epoch = nullptr;
    DevArray<BatchSlot> d_slots;
    DevArray<BatchWork> d_cs;
    // FD work lists per equilibrium order: 64 x 32 tiles (the first
    // Runge-Kutta stage, whose tiles index the fused diagnostics) and 64 x 16
    // tiles; the later stages take the list of the tile height chosen for
    // their order (rows per thread 4: 64 x 16, 8: 64 x 32)
    std::map<int, DevArray<BatchWork>> d_fd, d_fd16;
    std::map<int, int> n_fd, n_fd16;
    std::map<int, int> later_rows;  // tuned per order, kept for the server's life
    int n_cs = 0;
    DevArray<int> d_ids;
    hipGraphExec_t step_graph = nullptr;

    // counters (read under mu)
    uint64_t next_id = 1;
    double n_submitted = 0, n_completed = 0, steps_launched = 0, busy_s = 0;
    size_t used_snapshot = 0;
    int running_snapshot = 0;

    void run();
    int admit(const Pending &p);
    int rebuild();
    hipError_t enqueue_step(hipStream_t st);
    hipError_t tune_order(int N);
    int launch_chunk();
    int wait_chunk();
    void drain();
    void fail_all(int rc);
    void finish(uint64_t id, uint64_t tag, int status, double t_submit, double t_admit, std::vector<double> rows,
                double nu_app);
};

void lb_server::finish(uint64_t id, uint64_t tag, int status, double t_submit, double t_admit,
                       std::vector<double> rows, double nu_app)
{
    lb_result r{};
    r.nu_app = nu_app;
    r.id = id;
    r.tag = tag;
    r.status = status;
    r.nsamples = (int)(rows.size() / 6);
    r.samples = nullptr;
    if (!rows.empty()) {
        r.samples = static_cast<double *>(std::malloc(rows.size() * sizeof(double)));
        if (r.samples)
            std::memcpy(r.samples, rows.data(), rows.size() * sizeof(double));
        else {
            r.nsamples = 0;
            r.status = LB_ENOMEM;
        }
    }
    r.t_submit = t_submit;
    r.t_admit = t_admit;
    r.t_finish = now_s(t0);
    std::lock_guard<std::mutex> lk(mu);
    done.push_back(r);
    n_completed += 1;
    cv_done.notify_all();
}

int lb_server::admit(const Pending &p)
{
    const lb_request &q = p.req;
    lb_sim *sim = lb_create(q.model | LB_FP32, q.Nx, q.Ny, q.tau, q.dt, q.ds, q.N);
    if (!sim) return lb_last_error();
    // set up on the admission stream (each call synchronises only that
    // stream, not the chunk running on the compute stream), then step on the
    // compute stream
    int rc = lb_set_stream(sim, astream);
    if (rc == LB_OK) rc = lb_init(sim, q.rho, q.ux, q.uy);
    if (rc == LB_OK && q.ax) rc = lb_set_probe(sim, q.ax, q.ay, q.bx, q.by);
    if (rc == LB_OK) rc = lb_series_reserve(sim, q.nsteps / q.sample_every + 2);
    if (rc == LB_OK) rc = lb_set_stream(sim, stream);
    if (rc != LB_OK) {
        lb_destroy(sim);
        return rc;
    }
    Running r{};
    r.id = p.id;
    r.tag = q.tag;
    r.sim = sim;
    r.start_epoch = epoch;
    r.nsteps = q.nsteps;
    r.every = q.sample_every;
    r.t_submit = p.t_submit;
    r.t_admit = now_s(t0);
    r.footprint = p.footprint;
    r.nodes = p.nodes;
    r.N = sim->cs ? 0 : sim->N;
    r.dt = q.dt;
    r.decay_k2 = q.decay_k2;
    r.decay_omega = q.decay_omega;
    running.push_back(r);
    return LB_OK;
}

int lb_server::rebuild()
{
    const int n = (int)running.size();
    std::vector<BatchSlot> slots(n);
    std::vector<BatchWork> cs;
    std::map<int, std::vector<BatchWork>> fd, fd16;
    std::vector<int> ids(n);
    for (int i = 0; i < n; ++i) {
        lb_sim *s = running[i].sim;
        BatchSlot &b = slots[i];
        b.p = make_params<float>(s);
        for (int j = 0; j < 3; ++j) b.buf[j] = static_cast<float *>(s->buf[j]);
        b.partial = s->d_partial;
        b.series = s->d_series;
        if (s->probe) {
            b.ax = s->d_probe32;
            b.ay = s->d_probe32 + s->Nx;
            b.bx = s->d_probe32 + s->Nx + s->Ny;
            b.by = s->d_probe32 + 2 * s->Nx + s->Ny;
        } else {
            b.ax = b.ay = b.bx = b.by = nullptr;
        }
        b.model = s->cs ? 0 : 1;
        b.start_epoch = running[i].start_epoch;
        b.nsteps = running[i].nsteps;
        b.every = running[i].every;
        b.diag_blocks = diag_blocks_fused(s);
        b.tiles_x = (s->Nx + 63) / 64;
        ids[i] = i;
        if (s->cs) {
            for (int y = 0; y < s->Ny; ++y) cs.push_back({i, y});
        } else {
            const int tiles = fd_diag_blocks(s->Nx, s->Ny);
            auto &v = fd[s->N];
            for (int t = 0; t < tiles; ++t) v.push_back({i, t});
            auto &v16 = fd16[s->N];
            const int tiles16 = b.tiles_x * ((s->Ny + 15) / 16);
            for (int t = 0; t < tiles16; ++t) v16.push_back({i, t});
        }
    }
    hipError_t e = d_slots.ensure(std::max(n, 1));
    if (e == hipSuccess) e = d_ids.ensure(std::max(n, 1));
    if (e == hipSuccess) e = d_cs.ensure(std::max<size_t>(cs.size(), 1));
    if (e == hipSuccess && n > 0)
        e = hipMemcpyAsync(d_slots.ptr, slots.data(), n * sizeof(BatchSlot), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(d_ids.ptr, ids.data(), n * sizeof(int), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && !cs.empty())
        e = hipMemcpyAsync(d_cs.ptr, cs.data(), cs.size() * sizeof(BatchWork), hipMemcpyHostToDevice, stream);
    n_cs = (int)cs.size();
    auto upload_lists = [&](std::map<int, std::vector<BatchWork>> &lists, std::map<int, DevArray<BatchWork>> &dev,
                            std::map<int, int> &counts) {
        counts.clear();
        for (auto &kv : lists) {
            if (e != hipSuccess) break;
            auto &arr = dev[kv.first];
            e = arr.ensure(kv.second.size());
            if (e == hipSuccess)
                e = hipMemcpyAsync(arr.ptr, kv.second.data(), kv.second.size() * sizeof(BatchWork),
                                   hipMemcpyHostToDevice, stream);
            counts[kv.first] = (int)kv.second.size();
        }
    };
    upload_lists(fd, d_fd, n_fd);
    upload_lists(fd16, d_fd16, n_fd16);
    // the host vectors must outlive the copies
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    for (auto &kv : n_fd) {
        if (e != hipSuccess) break;
        if (!later_rows.count(kv.first)) e = tune_order(kv.first);
    }
    // capture one batched step of this running set
    if (step_graph) {
        (void)hipGraphExecDestroy(step_graph);
        step_graph = nullptr;
    }
    if (e == hipSuccess && use_graphs) {
        e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t ec = enqueue_step(stream);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(stream, &g);
            if (e == hipSuccess) e = ec;
            if (e == hipSuccess) e = hipGraphInstantiate(&step_graph, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
        }
    }
    return dev_status(e);
}

// The launches of one batched step, in the order of the single-simulation
// step (CS; per FD order the three Runge-Kutta stages), then the
// diagnostics sums and the step counter.
hipError_t lb_server::enqueue_step(hipStream_t st)
{
    hipError_t e = launch_cs_batch(d_slots.ptr, d_cs.ptr, n_cs, d_epoch, st);
    for (auto &kv : n_fd) {
        const int N = kv.first, rows = later_rows.count(N) ? later_rows[N] : 4;
        const BatchWork *later = rows == 8 ? d_fd[N].ptr : d_fd16[N].ptr;
        const int nlater = rows == 8 ? kv.second : n_fd16[N];
        // stage 1 always on the canonical 64 x 32 tiles of the fused diagnostics
        if (e == hipSuccess) e = launch_fd_batch(d_slots.ptr, d_fd[N].ptr, kv.second, N, 1, 8, d_epoch, st);
        for (int stage = 2; stage <= 3 && e == hipSuccess; ++stage)
            e = launch_fd_batch(d_slots.ptr, later, nlater, N, stage, rows, d_epoch, st);
    }
    if (e == hipSuccess) e = launch_finalize_batch(d_slots.ptr, d_ids.ptr, (int)running.size(), d_epoch, st);
    if (e == hipSuccess) e = launch_epoch_advance(d_epoch, st);
    return e;
}

// Later-stage tile height of FD order N: time the stage-2 launch over the
// current work list with 64 x 16 and with 64 x 32 tiles and keep the faster
// (the stage-2 output buffer is scratch between steps, so the timing leaves
// every state unchanged; results do not depend on the choice).
hipError_t lb_server::tune_order(int N)
{
    if (!tune_tiles) {
        later_rows[N] = 4;
        return hipSuccess;
    }
    // the two heights alternate launch by launch in the order 4 8 8 4 4 8 8 4,
    // an event between consecutive launches, so that both run under the same
    // shader clock (which drifts under sustained load and recovers when the
    // device idles) and neither is always the first of a pair
    constexpr int kReps = 4;
    auto launch = [&](int c) {
        const int rows = c ? 8 : 4;
        return launch_fd_batch(d_slots.ptr, rows == 8 ? d_fd[N].ptr : d_fd16[N].ptr, rows == 8 ? n_fd[N] : n_fd16[N],
                               N, 2, rows, d_epoch, stream);
    };
    hipEvent_t ev[2 * kReps + 1] = {};
    hipError_t e = hipSuccess;
    for (int i = 0; i <= 2 * kReps && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    for (int c = 0; c < 2 && e == hipSuccess; ++c) e = launch(c);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(ev[0], stream);
    auto which = [](int j) { return (j ^ (j >> 1)) & 1; };
    for (int j = 0; j < 2 * kReps && e == hipSuccess; ++j) {
        e = launch(which(j));
        if (e == hipSuccess) e = hipEventRecord(ev[j + 1], stream);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[2 * kReps]);
    float t[2] = {0.0f, 0.0f};
    for (int j = 0; j < 2 * kReps && e == hipSuccess; ++j) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, ev[j], ev[j + 1]);
        t[which(j)] += ms;
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e == hipSuccess) later_rows[N] = t[1] < t[0] ? 8 : 4;
    return e;
}

// Launch the next chunk of batched steps (asynchronously; chunk_done marks
// its end).
int lb_server::launch_chunk()
{
    int g = chunk;
    for (const Running &r : running) g = std::min(g, r.nsteps - (epoch - r.start_epoch));
    g = std::max(g, 1);
    hipError_t e = hipSuccess;
    for (int i = 0; i < g && e == hipSuccess; ++i) e = step_graph ? hipGraphLaunch(step_graph, stream) : enqueue_step(stream);
    if (e == hipSuccess) e = hipEventRecord(chunk_done, stream);
    if (e != hipSuccess) return dev_status(e);
    epoch += g;
    in_flight = true;
    std::lock_guard<std::mutex> lk(mu);
    steps_launched += g;
    return LB_OK;
}

int lb_server::wait_chunk()
{
    if (!in_flight) return LB_OK;
    in_flight = false;
    return dev_status(hipEventSynchronize(chunk_done));
}

void lb_server::drain()
{
    std::vector<Running> keep;
    for (Running &r : running) {
        if (epoch - r.start_epoch < r.nsteps) {
            keep.push_back(r);
            continue;
        }
        lb_sim *s = r.sim;
        // the batched steps advanced the handle's state
        s->steps = r.nsteps;
        if (s->cs) s->cur = r.nsteps & 1;
        s->series_t.clear();
        s->series_fused.clear();
        for (int t = 0; t < r.nsteps; t += r.every) {
            s->series_t.push_back(t);
            s->series_fused.push_back(1);
        }
        std::vector<double> rows(6 * (s->series_t.size() + 1));
        int got = lb_series_read(s, rows.data(), (int)s->series_t.size());
        int status = got >= 0 ? LB_OK : got;
        double fin[kDiag];
        if (status == LB_OK) status = lb_reduce(s, fin);
        double nu = std::nan("");
        if (status == LB_OK) {
            rows.resize(6 * ((size_t)got + 1));
            rows[6 * got] = (double)r.nsteps;
            for (int j = 0; j < kDiag; ++j) rows[6 * got + 1 + j] = fin[j];
            if (r.decay_k2 > 0.0) {
                // apparent viscosity: decay rate of the amplitude A against
                // t = step dt over every sample, over decay_k2
                const int n = got + 1;
                std::vector<double> t(n), amp(n);
                for (int i = 0; i < n; ++i) {
                    t[i] = rows[6 * i] * r.dt;
                    amp[i] = rows[6 * i + 5];
                }
                double rate = 0.0;
                if (fit_decay_rate(t.data(), amp.data(), n, r.decay_omega, &rate) == LB_OK) nu = rate / r.decay_k2;
            }
        } else {
            rows.clear();
        }
        lb_destroy(s);
        used -= r.footprint;
        nodes_in -= r.nodes;
        finish(r.id, r.tag, status, r.t_submit, r.t_admit, std::move(rows), nu);
    }
    running.swap(keep);
}

void lb_server::fail_all(int rc)
{
    // a device error ends every running request
    (void)hipStreamSynchronize(stream);
    in_flight = false;
    for (Running &r : running) {
        lb_destroy(r.sim);
        used -= r.footprint;
        nodes_in -= r.nodes;
        finish(r.id, r.tag, rc, r.t_submit, r.t_admit, {}, std::nan(""));
    }
    running.clear();
}

void lb_server::run()
{
    (void)hipSetDevice(device);
    bool changed = false;
    while (!stop.load()) {
        std::vector<Pending> admit_now;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (policy == 1 && queue.size() > 1)
                // smallest estimated work first; equal work in arrival order
                std::stable_sort(queue.begin(), queue.end(),
                                 [](const Pending &a, const Pending &b) { return a.work < b.work; });
            while (!queue.empty() && (int)(running.size() + admit_now.size()) < max_slots &&
                   used + queue.front().footprint <= budget &&
                   (node_limit == 0 || running.size() + admit_now.size() == 0 ||
                    nodes_in + queue.front().nodes <= node_limit)) {
                used += queue.front().footprint;
                nodes_in += queue.front().nodes;
                admit_now.push_back(queue.front());
                queue.pop_front();
            }
            if (running.empty() && admit_now.empty() && !in_flight) {
                used_snapshot = used;
                running_snapshot = 0;
                cv_work.wait_for(lk, std::chrono::milliseconds(5));
                continue;
            }
        }
        // 1. new simulations, set up while the chunk in flight runs
        for (const Pending &p : admit_now) {
            const int rc = admit(p);
            if (rc != LB_OK) {
                used -= p.footprint;
                nodes_in -= p.nodes;
                finish(p.id, p.req.tag, rc, p.t_submit, now_s(t0), {}, std::nan(""));
            } else {
                changed = true;
            }
        }
        const double tb = now_s(t0);
        // 2. the chunk in flight, and the simulations it finished
        int rc = wait_chunk();
        if (rc != LB_OK) {
            fail_all(rc);
            continue;
        }
        const size_t before = running.size();
        drain();
        if (running.size() != before) changed = true;
        // 3. descriptors and step graph of the new running set; 4. next chunk
        if (!running.empty()) {
            if (changed) rc = rebuild();
            changed = false;
            if (rc == LB_OK) rc = launch_chunk();
            if (rc != LB_OK) {
                fail_all(rc);
                continue;
            }
        }
        std::lock_guard<std::mutex> lk(mu);
        busy_s += now_s(t0) - tb;
        used_snapshot = used;
        running_snapshot = (int)running.size();
    }
    (void)wait_chunk();
}

extern "C" {

lb_server *lb_server_create(size_t hbm_budget_bytes, int max_slots, int chunk_steps)
{
    if (hbm_budget_bytes == 0 || max_slots < 1 || max_slots > 4096 || chunk_steps < 1) {
        set_last_error(LB_EINVAL);
        return nullptr;
    }
    lb_server *s = new (std::nothrow) lb_server();
    if (!s) {
        set_last_error(LB_ENOMEM);
        return nullptr;
    }
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->chunk = chunk_steps;
    s->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&s->device) != hipSuccess ||
        hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->astream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->chunk_done, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&s->d_epoch, sizeof(int)) != hipSuccess ||
        hipMemcpy(s->d_epoch, &s->epoch, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        if (s->d_epoch) (void)hipFree(s->d_epoch);
        if (s->chunk_done) (void)hipEventDestroy(s->chunk_done);
        if (s->astream) (void)hipStreamDestroy(s->astream);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        delete s;
        set_last_error(LB_EDEVICE);
        return nullptr;
    }
    return s;
}

int lb_server_configure(lb_server *s, int use_graphs, int tune_tiles)
{
    if (!s || (use_graphs != 0 && use_graphs != 1) || (tune_tiles != 0 && tune_tiles != 1))
        return set_last_error(LB_EINVAL);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->started.load()) return set_last_error(LB_ESTATE);
    s->use_graphs = use_graphs != 0;
    s->tune_tiles = tune_tiles != 0;
    return LB_OK;
}

int lb_server_set_policy(lb_server *s, int policy)
{
    if (!s || (policy != LB_ADMIT_ARRIVAL && policy != LB_ADMIT_SHORTEST)) return set_last_error(LB_EINVAL);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->started.load()) return set_last_error(LB_ESTATE);
    s->policy = policy;
    return LB_OK;
}

int lb_server_set_node_limit(lb_server *s, size_t max_nodes)
{
    if (!s) return set_last_error(LB_EINVAL);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->started.load()) return set_last_error(LB_ESTATE);
    s->node_limit = max_nodes;
    return LB_OK;
}

int lb_server_submit(lb_server *s, const lb_request *req, uint64_t *id)
{
    if (!s || !req || !req->rho || !req->ux || !req->uy || req->nsteps < 1 || req->sample_every < 1 ||
        (req->model & ~0xff) != 0)
        return set_last_error(LB_EINVAL);
    const bool probe_any = req->ax || req->ay || req->bx || req->by;
    const bool probe_all = req->ax && req->ay && req->bx && req->by;
    if (probe_any && !probe_all) return set_last_error(LB_EINVAL);
    if (!(req->decay_k2 >= 0.0) || !std::isfinite(req->decay_k2) || !(req->decay_omega >= 0.0) ||
        !std::isfinite(req->decay_omega) || (req->decay_k2 > 0.0 && !probe_all))
        return set_last_error(LB_EINVAL);
    const int rc = validate_create(req->model | LB_FP32, req->Nx, req->Ny, req->tau, req->dt, req->ds, req->N);
    if (rc != LB_OK) return set_last_error(rc);
    ModelInfo mi{};
    model_info(req->model, req->ds, req->dt, &mi);
    Pending p{};
    p.req = *req;
    p.footprint = footprint_of(*req, mi);
    p.nodes = (size_t)req->Nx * (size_t)req->Ny;
    // cost per node-step relative to a CS D2Q9 step: an FD step (three
    // WENO-5 stages) over K populations costs ~0.75 K of them (12 for D2Q16,
    // as the measured rates of the two kernels)
    p.work = (double)p.nodes * (double)req->nsteps * (req->model == LB_CS_D2Q9 ? 1.0 : 0.75 * mi.K);
    if (p.footprint > s->budget) return set_last_error(LB_EBUSY);
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->started.exchange(true)) s->worker = std::thread([s] { s->run(); });
    p.id = s->next_id++;
    p.t_submit = now_s(s->t0);
    s->queue.push_back(p);
    s->n_submitted += 1;
    s->cv_work.notify_all();
    if (id) *id = p.id;
    return LB_OK;
}

int lb_server_poll(lb_server *s, lb_result *out, int max, int timeout_us)
{
    if (!s || (max > 0 && !out) || max < 0) return set_last_error(LB_EINVAL);
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && timeout_us > 0)
        s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [s] { return !s->done.empty(); });
    int n = 0;
    while (n < max && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    return n;
}

void lb_server_release(lb_server *, lb_result *res)
{
    if (!res) return;
    std::free(res->samples);
    res->samples = nullptr;
    res->nsamples = 0;
}

double lb_server_clock(const lb_server *s) { return s ? now_s(s->t0) : -1.0; }

int lb_server_stats(const lb_server *s, double out[7])
{
    if (!s || !out) return set_last_error(LB_EINVAL);
    auto *m = const_cast<lb_server *>(s);
    std::lock_guard<std::mutex> lk(m->mu);
    out[0] = m->n_submitted;
    out[1] = m->n_completed;
    out[2] = (double)m->queue.size();
    out[3] = (double)m->running_snapshot;
    out[4] = (double)m->used_snapshot;
    out[5] = m->steps_launched;
    out[6] = m->busy_s;
    return LB_OK;
}

void lb_server_destroy(lb_server *s)
{
    if (!s) return;
    s->stop.store(true);
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->device);
    for (Running &r : s->running) lb_destroy(r.sim);
    s->running.clear();
    s->d_slots.release();
    s->d_cs.release();
    for (auto &kv : s->d_fd) kv.second.release();
    for (auto &kv : s->d_fd16) kv.second.release();
    s->d_ids.release();
    if (s->step_graph) (void)hipGraphExecDestroy(s->step_graph);
    if (s->d_epoch) (void)hipFree(s->d_epoch);
    if (s->chunk_done) (void)hipEventDestroy(s->chunk_done);
    for (lb_result &r : s->done) std::free(r.samples);
    if (s->astream) (void)hipStreamDestroy(s->astream);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
