// Job scheduler, serving loop and batch runner of libpps.
//
// Jobs of different kind, size, step count and lambda are admitted in FIFO
// order while arena memory and active slots allow, then their tiles are packed
// into epochs of a target GPU time.  Up to two epochs are in flight, on two
// streams: while the GPU runs epoch e the host plans e + 1 and admits new
// arrivals, so requests that arrive while others run join the next epoch, and
// e + 1's simulation starts as soon as e's ends, beside e's finalisation.  A
// job's finalisation (ABC select / compaction / moments, or the copy-out of a
// p-value tally) rides in the epoch that holds its last tile.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pps.h"
#include "pps_engine.hpp"
#include "pps_runtime.hpp"

namespace pps {

static double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

static uint64_t round256(uint64_t v) { return (v + 255) & ~static_cast<uint64_t>(255); }

// First-fit allocator over [0, size) of the caller's arena.
class ArenaAlloc {
  public:
    void init(uint64_t size)
    {
        size_ = size;
        free_.clear();
        if (size)
            free_[0] = size;
    }
    bool alloc(uint64_t len, uint64_t *off)
    {
        len = round256(len);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= len) {
                *off = it->first;
                const uint64_t rest = it->second - len;
                const uint64_t at = it->first + len;
                free_.erase(it);
                if (rest)
                    free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t len)
    {
        len = round256(len);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += len;
                return;
            }
        }
        free_[off] = len;
    }
    uint64_t size() const { return size_; }

  private:
    uint64_t size_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

enum class JobState { QUEUED, ACTIVE, DONE };

struct Job {
    uint64_t id = 0;
    pps_job spec;
    JobState state = JobState::QUEUED;
    int n_summ = 0;
    uint64_t arena_off = 0, arena_len = 0;
    bool has_arena = false;
    uint64_t capacity = 0;  // ABC records kept
    JobDev row;             // template of the job's rows (whole-job fields)
    FinJob fin;             // ABC finalisation
    uint64_t n_tiles = 0, next_tile = 0;
    int cls = CLASS_PATH;        // simulation kernel class of the job's rows
    uint64_t cost_per_tile = 0;  // in logistic-step units (draw_cost)
    pps_job_result result;
};

// Bytes and layout of a job's arena block.
struct JobLayout {
    uint64_t scratch = 0, idx = 0, theta = 0, dist = 0, total = 0, capacity = 0;
};

static JobLayout job_layout(const pps_job &j)
{
    JobLayout L;
    if (j.kind == PPS_JOB_PVALUE) {
        L.total = 256;
        return L;
    }
    const uint64_t n = j.sampling.n_draws;
    L.capacity = j.eps_mode == PPS_EPS_TOP_FRACTION ? top_count(j.eps_or_frac, n) : j.capacity;
    L.scratch = 0;
    L.idx = round256(abc_scratch_bytes(n));
    L.theta = L.idx + round256(L.capacity * sizeof(uint64_t));
    L.dist = L.theta + round256(L.capacity * PPS_MAX_PARAMS * sizeof(float));
    L.total = L.dist + round256(L.capacity * sizeof(float));
    return L;
}

// Validates a job and returns its summary count in *n_summ.
static int validate_job(const pps_job *j, int *n_summ)
{
    if (!j)
        return fail(PPS_EINVAL, "job is NULL");
    int rc = validate_model(&j->model, n_summ);
    if (rc != PPS_OK)
        return rc;
    if ((rc = validate_sampling(&j->sampling)) != PPS_OK)
        return rc;
    if (j->kind == PPS_JOB_ABC)
        return validate_abc(&j->model, j->y_obs, *n_summ, &j->sampling, j->eps_mode,
                            j->eps_or_frac);
    if (j->kind != PPS_JOB_PVALUE)
        return fail(PPS_EINVAL, "unknown job kind %d", j->kind);
    if (j->model.model != PPS_LOGISTIC_SDE && j->model.model != PPS_NORMAL_MEAN)
        return fail(PPS_EINVAL, "p-value jobs run the logistic SDE or normal-mean models");
    if (j->lambda_param < 0 || j->lambda_param >= j->model.n_params)
        return fail(PPS_EINVAL, "lambda_param %d out of range", j->lambda_param);
    pps_model m = j->model;
    m.prior[j->lambda_param].family = j->lambda_family;
    m.prior[j->lambda_param].b = j->lambda;
    int ns2 = 0;
    if (validate_model(&m, &ns2) != PPS_OK)
        return fail(PPS_EINVAL, "lambda %g gives an invalid prior", j->lambda);
    if (std::isnan(j->t_obs))
        return fail(PPS_EINVAL, "t_obs is NaN");
    return PPS_OK;
}

// The scheduler proper (no thread); the server and the batch runner drive it.
class Scheduler {
  public:
    // `engine` must have two slots and outlive the scheduler.
    void init(const pps_server_config &cfg, EpochEngine *engine, hipStream_t stream,
              bool no_release)
    {
        no_release_ = no_release;
        cfg_ = cfg;
        stream_ = stream;
        arena_.init(cfg.arena_bytes);
        plain_ = cfg.policy == PPS_POLICY_PLAIN;
        eng_ = engine;
    }

    // Takes ownership of a validated job and queues it.
    void enqueue(std::unique_ptr<Job> j)
    {
        queue_.push_back(j.get());
        jobs_[j->id] = std::move(j);
    }

    // One round: harvest finished epochs, admit, plan and launch.  With
    // `block` it waits for the oldest epoch when nothing else can be done.
    // *progress tells whether an epoch finished or was launched.  Returns
    // PPS_OK, or an error from the device.
    int step(bool block, bool *progress = nullptr)
    {
        const uint64_t harvested0 = harvested_;
        int rc = harvest(false);
        if (rc != PPS_OK)
            return rc;
        admit();
        bool launched = false;
        if (can_launch()) {
            rc = plan_and_launch(&launched);
            if (rc != PPS_OK)
                return rc;
        }
        if (!launched && block && !inflight_.empty())
            rc = harvest(true);
        if (progress)
            *progress = launched || harvested_ != harvested0;
        return rc;
    }

    // Waits for the epochs in flight and harvests them; admits and plans
    // nothing.  Returns the first error met, else PPS_OK.
    int drain()
    {
        int first = PPS_OK;
        while (!inflight_.empty()) {
            const int rc = harvest(true);
            if (rc != PPS_OK && first == PPS_OK)
                first = rc;
        }
        return first;
    }

    // Completes every job that has not finished with `status` (after an
    // error nothing more is planned, so no such job would ever finish).
    // Call after drain(): no epoch is in flight.
    void fail_pending(int status)
    {
        for (Job *j : queue_)
            complete(j, status);
        queue_.clear();
        for (Job *j : active_)
            if (j->state != JobState::DONE)
                complete(j, status);
        active_.clear();
    }

    // Host-side fault injection for tests of the error path: the harvest of
    // every epoch after the first `after_epochs` reports `status` in place of
    // its result (the epoch itself still runs to its end on the device).
    void inject_error(uint64_t after_epochs, int status)
    {
        inject_after_ = after_epochs;
        inject_status_ = status;
    }

    bool idle() const { return queue_.empty() && active_.empty() && inflight_.empty(); }
    bool has_inflight() const { return !inflight_.empty(); }
    bool can_plan() const
    {
        for (const Job *j : active_)
            if (j->next_tile < j->n_tiles)
                return true;
        return false;
    }

    Job *find(uint64_t id)
    {
        auto it = jobs_.find(id);
        return it == jobs_.end() ? nullptr : it->second.get();
    }
    void erase(uint64_t id)
    {
        Job *j = find(id);
        if (!j)
            return;
        if (j->has_arena)
            arena_.release(j->arena_off, j->arena_len);
        jobs_.erase(id);
    }
    size_t queued() const { return queue_.size(); }
    size_t active() const { return active_.size(); }
    uint64_t epochs() const { return epochs_; }
    double busy_s() const { return busy_s_; }
    uint64_t completed() const { return completed_; }
    const std::vector<double> &latencies() const { return latencies_; }
    void set_rate(double r) { rate_ = r; }
    double rate() const { return rate_; }

  private:
    struct InFlight {
        int slot;
        std::vector<Job *> finishing;
        std::vector<int> fin_index;     // ABC: index in the slot's results
        std::vector<uint32_t> count_at; // p-value: index in the slot's counts
        uint64_t cost;  // logistic-step units planned
    };

    bool can_launch() const
    {
        if (plain_)
            return inflight_.empty();
        return inflight_.size() < static_cast<size_t>(eng_->n_slots());
    }

    void complete(Job *j, int status)
    {
        j->state = JobState::DONE;
        j->result.status = status;
        j->result.t_done = now_s();
        ++completed_;
        latencies_.push_back(j->result.t_done - j->result.t_submit);
    }

    void admit()
    {
        while (!queue_.empty() && active_.size() < static_cast<size_t>(cfg_.max_active)) {
            Job *j = queue_.front();
            const JobLayout L = job_layout(j->spec);
            if (L.total > arena_.size()) {
                queue_.pop_front();
                fail(PPS_ENOMEM, "job %llu needs %llu arena bytes, the arena has %llu",
                     static_cast<unsigned long long>(j->id),
                     static_cast<unsigned long long>(L.total),
                     static_cast<unsigned long long>(arena_.size()));
                complete(j, PPS_ENOMEM);
                continue;
            }
            uint64_t off = 0;
            if (!arena_.alloc(L.total, &off)) {
                if (no_release_ && active_.empty() && inflight_.empty()) {
                    // batch mode keeps finished jobs' records: nothing will
                    // ever free this memory
                    queue_.pop_front();
                    fail(PPS_ENOMEM, "job %llu does not fit in the arena left by earlier jobs",
                         static_cast<unsigned long long>(j->id));
                    complete(j, PPS_ENOMEM);
                    continue;
                }
                break;  // FIFO: wait for memory to free up
            }
            queue_.pop_front();
            j->has_arena = true;
            j->arena_off = off;
            j->arena_len = L.total;
            j->capacity = L.capacity;
            j->result.t_admit = now_s();
            build_rows(j, L);
            j->state = JobState::ACTIVE;
            active_.push_back(j);
        }
    }

    void build_rows(Job *j, const JobLayout &L)
    {
        char *base = static_cast<char *>(cfg_.arena) + j->arena_off;
        const pps_job &s = j->spec;
        JobDev &row = j->row;
        if (s.kind == PPS_JOB_ABC) {
            const AbcScratch scr = abc_scratch_at(base + L.scratch, s.sampling.n_draws);
            fill_job(row, &s.model, &s.sampling, j->n_summ, JOB_WRITE_DIST);
            for (int k = 0; k < j->n_summ; ++k)
                row.y_obs[k] = static_cast<float>(s.y_obs[k]);
            row.dist = scr.dist;
            uint64_t *idx = reinterpret_cast<uint64_t *>(base + L.idx);
            float *theta = reinterpret_cast<float *>(base + L.theta);
            float *dist = reinterpret_cast<float *>(base + L.dist);
            fill_fin(j->fin, row, s.eps_mode, s.eps_or_frac, L.capacity, idx, theta, dist, scr);
            j->result.acc_idx = idx;
            j->result.acc_theta = theta;
            j->result.acc_dist = dist;
        } else {
            pps_model m = s.model;
            m.prior[s.lambda_param].family = s.lambda_family;
            m.prior[s.lambda_param].b = s.lambda;
            fill_job(row, &m, &s.sampling, j->n_summ, JOB_TALLY_STAT);
            row.t_obs = s.t_obs;
            row.counts = reinterpret_cast<unsigned long long *>(base);
            row.n_counts = 1;
        }
        j->cls = s.kind == PPS_JOB_ABC ? model_class(&s.model) : CLASS_PATH;
        j->n_tiles = eng_->tiles_for(j->cls, s.sampling.n_draws);
        j->next_tile = 0;
        j->cost_per_tile = eng_->tile_size(j->cls) * draw_cost(j->cls, row);
    }

    // Cost of one draw in units of one logistic-SDE Euler step of the whole
    // machine, from the classes' measured throughputs: a GARCH step costs
    // about 2.5, a toggle-switch cell-step 3.3, a tuberculosis event 2700 (its
    // run is one serial chain per workgroup), and a tuberculosis run takes
    // about 1.5 n_stop events.  The epoch budget and the measured rate are in
    // these units, so epochs of any mix of classes take about epoch_ms.
    static uint64_t draw_cost(int cls, const JobDev &row)
    {
        const uint64_t steps = static_cast<uint64_t>(row.steps > 0 ? row.steps : 1);
        const uint64_t cells = static_cast<uint64_t>(row.n_cells > 0 ? row.n_cells : 1);
        switch (cls) {
        case CLASS_GARCH:
            return (steps * 5 + 1) / 2;
        case CLASS_CELLS:
            return (cells * steps * 10 + 2) / 3;
        case CLASS_GILLESPIE:
            return cells * 4050;
        default:
            return steps;
        }
    }

    int plan_and_launch(bool *launched)
    {
        *launched = false;
        if (!can_plan())
            return PPS_OK;
        EpochPlan plan;
        InFlight fl;
        fl.cost = 0;
        double budget = cfg_.epoch_ms * 1e-3 * rate_;
        std::vector<std::pair<uint64_t, size_t>> order;  // (cost per tile, row index)
        std::vector<JobDev> rows;
        std::vector<Job *> row_job;
        for (Job *j : active_) {
            if (j->next_tile >= j->n_tiles)
                continue;
            if (!plain_ && budget <= 0.0)
                break;
            const uint64_t left = j->n_tiles - j->next_tile;
            uint64_t take = left;
            if (!plain_) {
                const double fit = std::floor(budget / static_cast<double>(j->cost_per_tile));
                take = fit < 1.0 ? 1 : std::min<uint64_t>(left, static_cast<uint64_t>(fit));
            }
            JobDev r = j->row;
            r.tile_offset = j->next_tile;
            r.n_tiles = take;
            const bool first = j->next_tile == 0;
            const bool last = j->next_tile + take == j->n_tiles;
            if (j->spec.kind == PPS_JOB_PVALUE) {
                r.row_flags = (first ? ROW_ZERO_COUNTS : 0u) | (last ? ROW_COPY_COUNTS : 0u);
            }
            j->next_tile += take;
            budget -= static_cast<double>(take * j->cost_per_tile);
            fl.cost += take * j->cost_per_tile;
            order.push_back({j->cost_per_tile, rows.size()});
            rows.push_back(r);
            row_job.push_back(j);
            if (last) {
                fl.finishing.push_back(j);
                if (j->spec.kind == PPS_JOB_ABC) {
                    fl.fin_index.push_back(static_cast<int>(plan.fins.size()));
                    plan.fins.push_back(j->fin);
                } else {
                    fl.fin_index.push_back(-1);
                }
            }
            if (plain_)
                break;  // one job per epoch
            if (rows.size() >= static_cast<size_t>(MAX_ROWS) ||
                plan.fins.size() >= static_cast<size_t>(MAX_FINS))
                break;
        }
        // Most expensive tiles first: the persistent grid drains in tile
        // order, so long tiles do not end up in the epoch's tail.
        std::stable_sort(order.begin(), order.end(),
                         [](const auto &a, const auto &b) { return a.first > b.first; });
        std::vector<Job *> ordered_job;
        // (rows keep this order within each class; p-value rows are all in
        // the path class, and ordered_job lists that class's jobs)
        for (const auto &o : order) {
            const int cls = row_job[o.second]->cls;
            plan.rows[cls].push_back(rows[o.second]);
            if (cls == CLASS_PATH)
                ordered_job.push_back(row_job[o.second]);
        }
        const int slot = free_slot();
        int rc = eng_->launch(slot, plan, eng_->slot_stream(slot, stream_));
        if (rc != PPS_OK)
            return rc;
        // Where each finishing p-value job's tally lands in the slot's counts.
        fl.count_at.assign(fl.finishing.size(), 0);
        for (size_t i = 0; i < fl.finishing.size(); ++i) {
            if (fl.finishing[i]->spec.kind != PPS_JOB_PVALUE)
                continue;
            for (size_t r = 0; r < ordered_job.size(); ++r)
                if (ordered_job[r] == fl.finishing[i] &&
                    (plan.rows[CLASS_PATH][r].row_flags & ROW_COPY_COUNTS))
                    fl.count_at[i] = plan.rows[CLASS_PATH][r].out_slot;
        }
        // finished jobs leave the active list when harvested; planned-out
        // jobs stay until then
        fl.slot = slot;
        inflight_.push_back(std::move(fl));
        ++epochs_;
        *launched = true;
        return PPS_OK;
    }

    int free_slot() const
    {
        for (int s = 0; s < eng_->n_slots(); ++s) {
            bool used = false;
            for (const InFlight &f : inflight_)
                used |= f.slot == s;
            if (!used)
                return s;
        }
        return 0;
    }

    // Harvests finished epochs in launch order.  With `wait` it blocks for
    // the oldest one.
    int harvest(bool wait)
    {
        while (!inflight_.empty()) {
            InFlight &f = inflight_.front();
            int rc = wait ? eng_->wait(f.slot) : eng_->poll(f.slot);
            if (rc == PPS_PENDING)
                return PPS_OK;
            if (rc == PPS_OK && inject_status_ != PPS_OK && harvested_ >= inject_after_)
                rc = fail(inject_status_, "injected error after %llu epochs",
                          static_cast<unsigned long long>(inject_after_));
            if (rc != PPS_OK) {
                for (Job *j : f.finishing) {
                    complete(j, rc);
                    active_.erase(std::find(active_.begin(), active_.end(), j));
                }
                inflight_.pop_front();
                ++harvested_;
                return rc;
            }
            const float ms = eng_->sim_ms(f.slot);
            if (ms > 0.0f) {
                busy_s_ += ms * 1e-3;
                const double r = static_cast<double>(f.cost) / (ms * 1e-3);
                if (f.cost > 0 && r > 0.0)
                    rate_ = 0.8 * rate_ + 0.2 * r;
            }
            const FinResult *fins = eng_->out_fin(f.slot);
            const unsigned long long *cnt = eng_->out_counts(f.slot);
            for (size_t i = 0; i < f.finishing.size(); ++i) {
                Job *j = f.finishing[i];
                pps_job_result &R = j->result;
                int status = PPS_OK;
                if (j->spec.kind == PPS_JOB_ABC) {
                    const FinResult &F = fins[f.fin_index[i]];
                    R.abc.n_accepted = F.n_accepted;
                    R.abc.eps_used = F.eps_used;
                    for (int p = 0; p < PPS_MAX_PARAMS; ++p) {
                        R.abc.mean[p] = F.mean[p];
                        R.abc.var[p] = F.var[p];
                    }
                    R.n_records = std::min<uint64_t>(F.n_accepted, j->capacity);
                    R.record_stride = j->capacity;
                    if (F.n_accepted > j->capacity)
                        status = PPS_ETRUNC;
                } else {
                    R.count_ge = cnt[f.count_at[i]];
                    R.pvalue = static_cast<double>(R.count_ge) /
                               static_cast<double>(j->spec.sampling.n_draws);
                }
                complete(j, status);
                active_.erase(std::find(active_.begin(), active_.end(), j));
            }
            inflight_.pop_front();
            ++harvested_;
            wait = false;
        }
        return PPS_OK;
    }

    pps_server_config cfg_;
    hipStream_t stream_ = nullptr;
    bool plain_ = false;
    bool no_release_ = false;
    ArenaAlloc arena_;
    EpochEngine *eng_ = nullptr;
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs_;
    std::deque<Job *> queue_;
    std::vector<Job *> active_;
    std::deque<InFlight> inflight_;
    uint64_t epochs_ = 0;
    uint64_t harvested_ = 0;
    uint64_t completed_ = 0;
    std::vector<double> latencies_;
    double busy_s_ = 0.0;
    double rate_ = 1.5e12;  // logistic-step units per second (updated from measurements)
    uint64_t inject_after_ = 0;
    int inject_status_ = PPS_OK;
};

static int validate_config(const pps_server_config *c)
{
    if (!c)
        return fail(PPS_EINVAL, "config is NULL");
    if (!c->arena || c->arena_bytes == 0)
        return fail(PPS_EINVAL, "an arena (device memory) is required");
    if (reinterpret_cast<uintptr_t>(c->arena) % 256 != 0)
        return fail(PPS_EINVAL, "the arena must be 256-byte aligned");
    if (c->max_active < 1 || c->max_active > 1024)
        return fail(PPS_EINVAL, "max_active must be in [1, 1024]");
    if (!(c->epoch_ms > 0.0))
        return fail(PPS_EINVAL, "epoch_ms must be > 0");
    if (c->policy != PPS_POLICY_BATCHED && c->policy != PPS_POLICY_PLAIN)
        return fail(PPS_EINVAL, "unknown policy %d", c->policy);
    return PPS_OK;
}

static std::unique_ptr<Job> make_job(const pps_job *spec, uint64_t id, int n_summ)
{
    std::unique_ptr<Job> j(new Job());
    j->id = id;
    j->spec = *spec;
    j->n_summ = n_summ;
    std::memset(&j->result, 0, sizeof j->result);
    j->result.kind = spec->kind;
    j->result.status = PPS_PENDING;
    j->result.t_submit = now_s();
    return j;
}

}  // namespace pps

using namespace pps;

struct pps_server {
    std::unique_ptr<EpochEngine> engine;
    Scheduler sched;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::unique_ptr<Job>> inbox;
    std::thread thread;
    bool stop = false;
    int error = PPS_OK;
    uint64_t next_id = 1;
    uint64_t submitted = 0;
    pps_server_config cfg;
    hipStream_t own_stream = nullptr;
    int device = 0;

    void run()
    {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (!stop) {
            while (!inbox.empty()) {
                sched.enqueue(std::move(inbox.front()));
                inbox.pop_front();
            }
            bool progress = false;
            int rc = sched.step(false, &progress);
            if (rc != PPS_OK) {
                error = rc;  // device error: stop serving
                break;
            }
            if (progress)
                continue;
            if (sched.has_inflight())
                // an epoch is running and nothing else can start: look again
                // in 25 us (a finished epoch's results wait at most that long
                // to become visible), or at once when a job is submitted
                cv.wait_for(lk, std::chrono::microseconds(25));
            else
                // idle, or waiting for arena memory: until a submission or release
                cv.wait(lk, [&] { return stop || !inbox.empty() || released; });
            released = false;
        }
        // Shutdown or error: wait for the epochs in flight only; nothing is
        // admitted or planned any more.
        const int rc = sched.drain();
        if (error == PPS_OK && rc != PPS_OK && !stop)
            error = rc;
        if (error != PPS_OK) {
            // every job that has not finished ends with the error, so that
            // pps_poll reports it instead of PPS_PENDING
            while (!inbox.empty()) {
                sched.enqueue(std::move(inbox.front()));
                inbox.pop_front();
            }
            sched.fail_pending(error);
        }
    }
    bool released = false;
};

extern "C" {

int64_t pps_job_arena_bytes(const pps_job *job)
{
    clear_error();
    int ns = 0;
    int rc = validate_job(job, &ns);
    if (rc != PPS_OK)
        return rc;
    return static_cast<int64_t>(job_layout(*job).total);
}

int pps_run_batch(const pps_job *jobs, int n_jobs, const pps_server_config *config,
                  pps_job_result *results)
{
    clear_error();
    int rc = validate_config(config);
    if (rc != PPS_OK)
        return rc;
    if (!jobs || n_jobs < 1 || !results)
        return fail(PPS_EINVAL, "jobs, n_jobs >= 1 and results are required");
    std::vector<int> n_summ(n_jobs);
    for (int i = 0; i < n_jobs; ++i)
        if ((rc = validate_job(&jobs[i], &n_summ[i])) != PPS_OK)
            return fail(rc, "job %d: %s", i, last_error());
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->batch_engine) {
        std::unique_ptr<EpochEngine> e(new EpochEngine());
        if ((rc = e->init(2, c->cu_count)) != PPS_OK)
            return rc;
        c->batch_engine = std::move(e);
    }
    for (int cls = 0; cls < N_CLASSES; ++cls)
        c->batch_engine->set_shape(cls, c->engine->shape(cls));
    Scheduler sched;
    sched.init(*config, c->batch_engine.get(), static_cast<hipStream_t>(config->stream), true);
    for (int i = 0; i < n_jobs; ++i)
        sched.enqueue(make_job(&jobs[i], static_cast<uint64_t>(i + 1), n_summ[i]));
    while (!sched.idle()) {
        if ((rc = sched.step(true)) != PPS_OK) {
            // wait for the other epoch in flight, then report the error as
            // the status of every job that did not finish
            sched.drain();
            sched.fail_pending(rc);
            for (int i = 0; i < n_jobs; ++i)
                results[i] = sched.find(static_cast<uint64_t>(i + 1))->result;
            return rc;
        }
    }
    for (int i = 0; i < n_jobs; ++i)
        results[i] = sched.find(static_cast<uint64_t>(i + 1))->result;
    return PPS_OK;
}

int pps_server_create(const pps_server_config *config, pps_server **server)
{
    clear_error();
    int rc = validate_config(config);
    if (rc != PPS_OK)
        return rc;
    if (!server)
        return fail(PPS_EINVAL, "server is NULL");
    Context *c = current_context(&rc);
    if (!c)
        return rc;
    std::unique_ptr<pps_server> s(new pps_server());
    s->cfg = *config;
    s->device = c->device;
    hipStream_t stream = static_cast<hipStream_t>(config->stream);
    if (!stream) {
        hipError_t e = hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking);
        if (e != hipSuccess)
            return fail_hip(e, "server stream");
        stream = s->own_stream;
    }
    s->engine.reset(new EpochEngine());
    if ((rc = s->engine->init(2, c->cu_count)) != PPS_OK)
        return rc;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        for (int cls = 0; cls < N_CLASSES; ++cls)
            s->engine->set_shape(cls, c->engine->shape(cls));
    }
    s->sched.init(*config, s->engine.get(), stream, false);
    pps_server *raw = s.get();
    s->thread = std::thread([raw] { raw->run(); });
    *server = s.release();
    return PPS_OK;
}

int pps_submit(pps_server *server, const pps_job *job, uint64_t *job_id)
{
    clear_error();
    if (!server || !job_id)
        return fail(PPS_EINVAL, "server and job_id are required");
    int ns = 0;
    int rc = validate_job(job, &ns);
    if (rc != PPS_OK)
        return rc;
    {
        std::lock_guard<std::mutex> lk(server->mu);
        if (server->error != PPS_OK)
            return fail(server->error, "server stopped after a device error");
        const size_t waiting = server->inbox.size() + server->sched.queued();
        if (server->cfg.queue_capacity > 0 &&
            waiting >= static_cast<size_t>(server->cfg.queue_capacity))
            return fail(PPS_EBUSY, "submission queue full (%zu waiting)", waiting);
        const uint64_t id = server->next_id++;
        server->inbox.push_back(make_job(job, id, ns));
        ++server->submitted;
        *job_id = id;
    }
    server->cv.notify_one();
    return PPS_OK;
}

int pps_poll(pps_server *server, uint64_t job_id, pps_job_result *out)
{
    clear_error();
    if (!server)
        return fail(PPS_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(server->mu);
    Job *j = server->sched.find(job_id);
    if (!j) {
        for (const auto &p : server->inbox)
            if (p->id == job_id)
                return server->error != PPS_OK
                           ? fail(server->error, "server stopped after an error")
                           : PPS_PENDING;
        return fail(PPS_ENOTFOUND, "unknown job %llu", static_cast<unsigned long long>(job_id));
    }
    if (j->state != JobState::DONE)
        return server->error != PPS_OK ? fail(server->error, "server stopped after an error")
                                       : PPS_PENDING;
    if (out)
        *out = j->result;
    return j->result.status;
}

int pps_release(pps_server *server, uint64_t job_id)
{
    clear_error();
    if (!server)
        return fail(PPS_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(server->mu);
    Job *j = server->sched.find(job_id);
    if (!j) {
        for (const auto &p : server->inbox)
            if (p->id == job_id)
                return fail(PPS_EBUSY, "job %llu has not started",
                            static_cast<unsigned long long>(job_id));
        return fail(PPS_ENOTFOUND, "unknown job %llu", static_cast<unsigned long long>(job_id));
    }
    if (j->state != JobState::DONE)
        return fail(PPS_EBUSY, "job %llu has not finished", static_cast<unsigned long long>(job_id));
    server->sched.erase(job_id);
    server->released = true;
    server->cv.notify_one();
    return PPS_OK;
}

int pps_server_stats_get(pps_server *server, pps_server_stats *stats)
{
    clear_error();
    if (!server || !stats)
        return fail(PPS_EINVAL, "server and stats are required");
    std::lock_guard<std::mutex> lk(server->mu);
    std::memset(stats, 0, sizeof *stats);
    stats->submitted = server->submitted;
    stats->completed = server->sched.completed();
    stats->epochs = server->sched.epochs();
    stats->queued = server->sched.queued() + server->inbox.size();
    stats->active = server->sched.active();
    stats->busy_s = server->sched.busy_s();
    std::vector<double> l = server->sched.latencies();
    if (!l.empty()) {
        std::sort(l.begin(), l.end());
        auto q = [&](double p) {
            const size_t k = static_cast<size_t>(std::ceil(p * static_cast<double>(l.size()))) - 1;
            return l[std::min(k, l.size() - 1)];
        };
        stats->latency_p50_s = q(0.50);
        stats->latency_p99_s = q(0.99);
    }
    return PPS_OK;
}

int pps_server_inject_error(pps_server *server, uint64_t after_epochs, int status)
{
    clear_error();
    if (!server)
        return fail(PPS_EINVAL, "server is NULL");
    if (status >= PPS_OK)
        return fail(PPS_EINVAL, "the injected status must be an error (< 0)");
    {
        std::lock_guard<std::mutex> lk(server->mu);
        server->sched.inject_error(after_epochs, status);
    }
    server->cv.notify_one();
    return PPS_OK;
}

int pps_server_destroy(pps_server *server)
{
    clear_error();
    if (!server)
        return fail(PPS_EINVAL, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(server->mu);
        server->stop = true;
    }
    server->cv.notify_all();
    if (server->thread.joinable())
        server->thread.join();
    hipStream_t own = server->own_stream;
    delete server;  // the engine waits for its epochs before freeing
    if (own)
        (void)hipStreamDestroy(own);
    return PPS_OK;
}

}  // extern "C"
