// Serving loop of the gpeval library: continuous batching of evaluation jobs.
//
// Jobs arrive through gp_server_submit at any time.  Host worker threads
// validate and compile each job's tree as it arrives.  A dispatcher admits
// compiled jobs in arrival order while the HBM budget and the number of
// in-flight batches allow, merges the admitted jobs that share a case set
// into one batch (one persistent launch for full jobs; one donor launch and
// one walk launch for incremental jobs) and enqueues it on one of several
// streams, so batches admitted while others run overlap on the device.  A
// completion thread waits for each batch, copies the results out and
// releases the batch's memory, except for full jobs kept resident as parents
// (their trees, records and values stay on the device for later incremental
// children until gp_server_release).  The paper's answer to uneven task
// sizes is to run more independent jobs than there are workers (Section
// 4.1); here the device runs several batches of jobs at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <thread>

#include "runtime.h"

namespace gpe {

namespace {

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct SBatch;

struct SJob {
    int64_t ticket = 0;
    int kind = GP_JOB_FULL;
    gp_handle cases_h = 0;
    std::shared_ptr<CaseSet> cs;
    std::vector<uint8_t> ops;               // prefix layout (converted on arrival)
    std::vector<int64_t> points;            // record points, prefix-converted (FULL)
    std::vector<int64_t> caller_points;     // as given (spine keys)
    int64_t parent_ticket = 0;
    int64_t point = 0;                      // caller's index (INCREMENTAL)
    bool keep_resident = false;
    int layout = GP_PREFIX;
    TreeProg prog;                          // FULL: compiled on arrival
    bool device_compiled = false;           // FULL: prog was built on the device
    uint64_t est_bytes = 0;
    enum State { ARRIVED, READY, RUNNING, DONE } state = ARRIVED;
    double t_submit = 0, t_ready = 0, t_admit = 0, t_enq = 0, t_done = 0;
    gp_job_result result{};
    std::vector<uint8_t> root;              // host copy of the output vector
    // resident parent (FULL + keep_resident, after completion)
    std::shared_ptr<struct ResidentBatch> rb;
    Pop* pop = nullptr;
    int64_t tree_in_pop = -1;
    // FULL + keep_resident: incremental children submitted and not done yet
    int64_t pending_children = 0;
};

// Memory of a finished full batch kept for its resident parents; returned
// to the budget when the last of them is released.
struct ResidentBatch {
    std::shared_ptr<Pop> pop;
    uint64_t bytes = 0;
    int refs = 0;
};

struct SBatch {
    int slot = 0;                           // stream slot
    int kind = GP_JOB_FULL;
    std::vector<std::shared_ptr<SJob>> jobs;
    std::vector<std::shared_ptr<SJob>> parents;   // INCREMENTAL: each job's resident parent
    std::shared_ptr<Pop> pop;               // FULL batches
    std::unique_ptr<IncOut> inc;            // INCREMENTAL batches
    hipEvent_t done_ev = nullptr;
    uint64_t bytes = 0;                     // charged against the server budget
    ~SBatch()
    {
        if (done_ev) (void)hipEventDestroy(done_ev);
    }
};

struct Server {
    Ctx* ctx = nullptr;
    gp_server_cfg cfg{};
    uint64_t budget = 0;
    std::map<TuneKey, Launch> tuned;
    int forced_variant = -1;
    int forced_waves = -1;

    std::mutex mu;
    std::condition_variable cv_prep, cv_disp, cv_done;
    bool stopping = false;
    int64_t next_ticket = 1;
    std::unordered_map<int64_t, std::shared_ptr<SJob>> jobs;
    std::deque<std::shared_ptr<SJob>> arrived;
    std::list<std::shared_ptr<SJob>> ready;     // arrival order
    std::deque<std::shared_ptr<SBatch>> inflight;
    std::vector<std::shared_ptr<SBatch>> graveyard;  // finished, memory not yet freed
    std::vector<char> slot_busy;
    uint64_t admitted_bytes = 0;

    std::vector<hipStream_t> streams;
    std::vector<hipStream_t> prep_streams;   // one per prep thread, for device compilation
    std::vector<std::unique_ptr<DevArena>> prep_arenas;   // and its temporaries
    int64_t device_compile_nodes = 0;        // FULL jobs this large compile on the device (0: never)
    std::vector<void*> pinned;               // per slot staging buffer
    size_t pinned_bytes = 0;
    std::vector<std::thread> workers;
    std::thread dispatcher, completer;
};

namespace {

int variant_for(Server* S, int vtype, const CaseSet* cs, const Pop* p)
{
    Variant* vt = variant_table();
    auto ok = [&](int v) {
        return v >= 0 && v < variant_count() &&
               variant_fits(vt[v], vtype, p->max_stack, p->n_inputs, cs->n_elems, cs->stride,
                            vtype == GP_BOOL ? 8 : 4);
    };
    if (ok(S->forced_variant)) return S->forced_variant;
    int wantK = vtype == GP_F32 ? (cs->n_elems <= 64 ? 1 : cs->n_elems <= 128 ? 2 : 4) : (cs->n_elems <= 64 ? 1 : 2);
    for (int v = 0; v < variant_count(); ++v)
        if (ok(v) && vt[v].K == wantK && vt[v].table) return v;
    for (int v = 0; v < variant_count(); ++v)
        if (ok(v) && vt[v].K == wantK) return v;
    for (int v = 0; v < variant_count(); ++v)
        if (ok(v)) return v;
    return -1;
}

uint64_t estimate_full(const TreeProg& pg, const CaseSet* cs)
{
    const uint64_t esz = cs->vtype == GP_BOOL ? 8 : 4;
    const uint64_t vec = (uint64_t)cs->stride * esz;
    uint64_t b = pg.code.size() * 4 + pg.chunks.size() * (32 + 16 + 8 * 4) + 4096;
    b += (pg.chunks.size() + 1) * vec + (uint64_t)pg.n_records * vec;
    for (auto& sp : pg.spines) b += sp.levels.size() * 16;
    return b + 64 * 1024;   // plan, graph-free launch state, fitness
}

// Workgroups a prep thread's compilation may use at once: a small slice of the
// device, which is busy with the batches in flight.
constexpr int kPrepBlocks = 32;

// Compile a FULL job's tree on the device, on its prep thread's stream st with
// that thread's arena for temporaries, into j->prog (host memory), so the job
// batches with the others exactly as a tree compiled on the host.
int compile_on_device(Server* S, SJob* j, hipStream_t st, DevArena* arena)
{
    Ctx* c = S->ctx;
    const CaseSet* cs = j->cs.get();
    const int64_t n = (int64_t)j->ops.size();
    int rc = arena_reset(c, arena);
    if (rc != GP_OK) return rc;
    DevBuf dops, doffs;
    rc = scratch_alloc(c, arena, dops, (size_t)n + 32);
    if (rc != GP_OK) return rc;
    rc = scratch_alloc(c, arena, doffs, 16);
    if (rc != GP_OK) return rc;
    const int64_t offs[2] = {0, n};
    if (hipMemcpyAsync(dops.p, j->ops.data(), (size_t)n, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(doffs.p, offs, 16, hipMemcpyHostToDevice, st) != hipSuccess)
        return set_err(c, GP_EDEVICE, "upload of a served tree failed");
    const int64_t np = (int64_t)j->points.size();
    const int64_t roffs[2] = {0, np};
    std::vector<TreeProg> progs;
    rc = device_compile_population(c, cs->vtype, cs->n_inputs, 1, dops.as<uint8_t>(), doffs.as<int64_t>(), offs,
                                   j->ops.data(), np ? j->points.data() : nullptr, np ? roffs : nullptr,
                                   np ? j->caller_points.data() : nullptr,
                                   auto_chunk_nodes(cs->vtype, n, 1, cs->T), 0, nullptr, &progs, arena, st,
                                   kPrepBlocks);
    if (rc != GP_OK) {
        (void)hipStreamSynchronize(st);        // nothing may still use the arena
        return rc;
    }
    j->prog = std::move(progs[0]);
    j->device_compiled = true;
    return GP_OK;
}

uint64_t estimate_incremental(int64_t donor_nodes, const CaseSet* cs)
{
    const uint64_t esz = cs->vtype == GP_BOOL ? 8 : 4;
    const uint64_t vec = (uint64_t)cs->stride * esz;
    return (uint64_t)donor_nodes * 4 + (donor_nodes / 64 + 2) * vec + 2 * vec + 64 * 1024;
}

// A child that reaches DONE no longer holds its parent (S->mu held).
void child_done(Server* S, SJob* j)
{
    if (j->kind != GP_JOB_INCREMENTAL) return;
    auto pit = S->jobs.find(j->parent_ticket);
    if (pit != S->jobs.end() && pit->second->pending_children > 0) --pit->second->pending_children;
}

void fail_job(Server* S, SJob* j, int code)
{
    j->result.status = code;
    j->state = SJob::DONE;
    j->t_done = now_ms();
    j->result.latency_ms = j->t_done - j->t_submit;
    child_done(S, j);
}

// ------------------------------------------------------------ workers
void prep_worker(Server* S, int idx)
{
    for (;;) {
        std::shared_ptr<SJob> j;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_prep.wait(lk, [&] { return S->stopping || !S->arrived.empty(); });
            if (S->stopping) return;
            j = S->arrived.front();
            S->arrived.pop_front();
        }
        int status = GP_OK;
        std::string why;
        const CaseSet* cs = j->cs.get();
        if (j->layout == GP_POSTFIX) {
            std::vector<uint8_t> pre;
            std::vector<int64_t> map;
            if (!postfix_to_prefix(j->ops.data(), (int64_t)j->ops.size(), cs->n_inputs, &pre, &map, &why)) {
                status = GP_EINVAL;
            } else {
                for (auto& q : j->points) q = (q >= 0 && q < (int64_t)map.size()) ? map[q] : -1;
                j->ops.swap(pre);
            }
        } else if (!validate_prefix(j->ops.data(), (int64_t)j->ops.size(), cs->n_inputs, &why)) {
            status = GP_EINVAL;
        }
        if (status == GP_OK && j->kind == GP_JOB_FULL && S->device_compile_nodes > 0 &&
            (int64_t)j->ops.size() >= S->device_compile_nodes) {
            status = compile_on_device(S, j.get(), S->prep_streams[idx], S->prep_arenas[idx].get());
            if (status == GP_OK) {
                for (size_t i = 0; i < j->caller_points.size(); ++i) j->prog.spines[i].point = j->caller_points[i];
                j->est_bytes = estimate_full(j->prog, cs);
            }
        } else if (status == GP_OK && j->kind == GP_JOB_FULL) {
            CompileOptions opt;
            opt.vtype = cs->vtype;
            opt.n_inputs = cs->n_inputs;
            opt.chunk_nodes = auto_chunk_nodes(cs->vtype, (int64_t)j->ops.size(), 1, cs->T);
            opt.stack_slots = compile_stack_slots();
            // a large tree is compiled on a few threads (its latency is mostly this)
            if (j->ops.size() >= 1000000) opt.threads = 4;
            if (!compile_tree(j->ops.data(), (int64_t)j->ops.size(), opt, j->points.data(), (int64_t)j->points.size(),
                              &j->prog, &why)) {
                status = GP_EINVAL;
            } else {
                for (size_t i = 0; i < j->caller_points.size(); ++i) j->prog.spines[i].point = j->caller_points[i];
                j->est_bytes = estimate_full(j->prog, cs);
            }
        } else if (status == GP_OK) {
            j->est_bytes = estimate_incremental((int64_t)j->ops.size(), cs);
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (status != GP_OK) {
                fail_job(S, j.get(), status);
                S->cv_done.notify_all();
            } else if (j->est_bytes > S->budget) {
                fail_job(S, j.get(), GP_EBUDGET);
                S->cv_done.notify_all();
            } else {
                j->state = SJob::READY;
                j->t_ready = now_ms();
                S->ready.push_back(j);
            }
        }
        S->cv_disp.notify_all();
    }
}

// Free finished batches once nothing is in flight (hipFree waits for the
// device).  Their bytes stay charged until then, so admission never counts
// on memory that is still allocated.
void collect_graveyard(Server* S, std::unique_lock<std::mutex>& lk)
{
    if (S->graveyard.empty() || !S->inflight.empty()) return;
    std::vector<std::shared_ptr<SBatch>> dead;
    dead.swap(S->graveyard);
    uint64_t freed = 0;
    for (auto& b : dead) freed += b->bytes;
    lk.unlock();
    dead.clear();
    lk.lock();
    S->admitted_bytes -= std::min(S->admitted_bytes, freed);
}

int launch_batch(Server* S, SBatch* b)
{
    Ctx* c = S->ctx;
    hipStream_t s = S->streams[b->slot];
    const std::shared_ptr<SJob>& j0 = b->jobs.front();
    const CaseSet* cs = j0->cs.get();
    const gp_handle ch = j0->cases_h;
    const size_t esz = cs->vtype == GP_BOOL ? 8 : 4;
    const size_t vbytes = (size_t)cs->n_elems * esz;
    const int64_t n = (int64_t)b->jobs.size();
    uint8_t* stage = (uint8_t*)S->pinned[b->slot];
    // staging layout: [n] fitness (8 B), [n] stop (4 B), [n] interp (8 B), [n][vbytes] roots
    uint8_t* st_fit = stage;
    uint8_t* st_stop = st_fit + 8 * n;
    uint8_t* st_int = st_stop + 4 * n;
    uint8_t* st_root = st_int + 8 * n;
    if (b->kind == GP_JOB_FULL) {
        std::vector<TreeProg> progs(n);
        std::vector<int64_t> nodes(n);
        for (int64_t i = 0; i < n; ++i) {
            progs[i] = std::move(b->jobs[i]->prog);
            nodes[i] = (int64_t)b->jobs[i]->ops.size();
        }
        b->pop = std::make_shared<Pop>();
        int rc0 = assemble_population(c, cs->vtype, cs->n_inputs, progs, nodes, 0, b->pop.get(), s);
        if (rc0 != GP_OK) return rc0;
        const Launch L{variant_for(S, cs->vtype, cs, b->pop.get()), std::max(0, S->forced_waves)};
        if (L.variant < 0) return GP_EINVAL;
        const int rc = enqueue_full(c, b->pop.get(), ch, cs, L, false, false, s, nullptr);
        if (rc != GP_OK) return rc;
        if (hipMemcpyAsync(st_fit, b->pop->fit.p, (size_t)n * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpy2DAsync(st_root, vbytes, b->pop->vecs.p, (size_t)cs->stride * esz, vbytes, n,
                             hipMemcpyDeviceToHost, s) != hipSuccess)
            return GP_EDEVICE;
    } else {
        std::vector<IncJob> ij(n);
        for (int64_t i = 0; i < n; ++i) {
            SJob* j = b->jobs[i].get();
            SJob* par = b->parents[i].get();
            ij[i] = IncJob{par->pop, par->tree_in_pop, j->point, j->ops.data(), (int64_t)j->ops.size()};
        }
        b->inc = std::make_unique<IncOut>();
        int rc = enqueue_incremental(c, ij, ch, cs, true, s, b->inc.get(), nullptr);
        if (rc != GP_OK) return rc;
        if (hipMemcpyAsync(st_fit, b->inc->fit.p, (size_t)n * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(st_stop, b->inc->stop.p, (size_t)n * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(st_int, b->inc->interp.p, (size_t)n * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpy2DAsync(st_root, vbytes, b->inc->root.p, (size_t)cs->stride * esz, vbytes, n,
                             hipMemcpyDeviceToHost, s) != hipSuccess)
            return GP_EDEVICE;
    }
    if (hipEventRecord(b->done_ev, s) != hipSuccess) return GP_EDEVICE;
    return GP_OK;
}

// Admit ready jobs in arrival order into one batch: same kind and case set,
// parents finished, within the budget and the batch size limit.
std::shared_ptr<SBatch> form_batch(Server* S, int slot)
{
    auto b = std::make_shared<SBatch>();
    b->slot = slot;
    const size_t stage_per_job = 20 + (size_t)16384 * 8;
    const int64_t max_jobs = std::min<int64_t>(S->cfg.max_batch_jobs, (int64_t)(S->pinned_bytes / stage_per_job));
    for (auto it = S->ready.begin(); it != S->ready.end() && (int64_t)b->jobs.size() < max_jobs;) {
        SJob* j = it->get();
        if (j->kind == GP_JOB_INCREMENTAL) {
            auto pit = S->jobs.find(j->parent_ticket);
            if (pit == S->jobs.end()) {
                // cannot happen while the child counts against its parent;
                // a child never waits for a parent that is gone
                fail_job(S, j, GP_ENOTFOUND);
                it = S->ready.erase(it);
                S->cv_done.notify_all();
                continue;
            }
            if (pit->second->state != SJob::DONE) {
                ++it;                          // parent not finished yet
                continue;
            }
            if (pit->second->result.status != GP_OK || !pit->second->rb) {
                fail_job(S, j, pit->second->result.status != GP_OK ? pit->second->result.status : GP_ENOTFOUND);
                it = S->ready.erase(it);
                S->cv_done.notify_all();
                continue;
            }
        }
        if (!b->jobs.empty() && (j->kind != b->kind || j->cases_h != b->jobs.front()->cases_h)) {
            ++it;
            continue;
        }
        if (S->admitted_bytes + b->bytes + j->est_bytes > S->budget) break;   // keep arrival order
        if (b->jobs.empty()) b->kind = j->kind;
        b->bytes += j->est_bytes;
        j->state = SJob::RUNNING;
        j->t_admit = now_ms();
        if (j->kind == GP_JOB_INCREMENTAL) b->parents.push_back(S->jobs.at(j->parent_ticket));
        b->jobs.push_back(*it);
        it = S->ready.erase(it);
    }
    if (b->jobs.empty()) return nullptr;
    return b;
}

void dispatch_loop(Server* S)
{
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        if (S->stopping) return;
        collect_graveyard(S, lk);
        int slot = -1;
        for (int i = 0; i < (int)S->slot_busy.size(); ++i)
            if (!S->slot_busy[i]) {
                slot = i;
                break;
            }
        std::shared_ptr<SBatch> b;
        if (slot >= 0 && !S->ready.empty()) b = form_batch(S, slot);
        if (!b) {
            S->cv_disp.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        S->slot_busy[slot] = 1;
        S->admitted_bytes += b->bytes;
        if (b->done_ev == nullptr) (void)hipEventCreateWithFlags(&b->done_ev, hipEventDisableTiming);
        lk.unlock();
        int rc = launch_batch(S, b.get());
        lk.lock();
        if (rc != GP_OK) {
            for (auto& j : b->jobs) fail_job(S, j.get(), rc);
            S->cv_done.notify_all();
            (void)hipStreamSynchronize(S->streams[slot]);
            S->slot_busy[slot] = 0;
            S->graveyard.push_back(b);
            continue;
        }
        const double t_enq = now_ms();
        for (auto& j : b->jobs) j->t_enq = t_enq;
        S->inflight.push_back(b);
        S->cv_done.notify_all();
    }
}

void complete_loop(Server* S)
{
    (void)hipSetDevice(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_done.wait(lk, [&] { return S->stopping || !S->inflight.empty(); });
        if (S->inflight.empty() && S->stopping) return;
        // wait for whichever in-flight batch finishes first
        std::shared_ptr<SBatch> b;
        while (!b) {
            for (auto it = S->inflight.begin(); it != S->inflight.end(); ++it)
                if (hipEventQuery((*it)->done_ev) == hipSuccess) {
                    b = *it;
                    S->inflight.erase(it);
                    break;
                }
            if (!b) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(50));
                lk.lock();
            }
        }
        const double t = now_ms();
        const std::shared_ptr<SJob> j0 = b->jobs.front();
        const CaseSet* cs = j0->cs.get();
        const size_t esz = cs->vtype == GP_BOOL ? 8 : 4;
        const size_t vbytes = (size_t)cs->n_elems * esz;
        const int64_t n = (int64_t)b->jobs.size();
        const uint8_t* stage = (const uint8_t*)S->pinned[b->slot];
        const uint8_t* st_fit = stage;
        const uint8_t* st_stop = st_fit + 8 * n;
        const uint8_t* st_int = st_stop + 4 * n;
        const uint8_t* st_root = st_int + 8 * n;
        for (int64_t i = 0; i < n; ++i) {
            SJob* j = b->jobs[i].get();
            if (cs->vtype == GP_BOOL) std::memcpy(&j->result.fitness_i64, st_fit + 8 * i, 8);
            else std::memcpy(&j->result.fitness_f64, st_fit + 8 * i, 8);
            j->root.assign(st_root + vbytes * i, st_root + vbytes * (i + 1));
            if (b->kind == GP_JOB_INCREMENTAL) {
                std::memcpy(&j->result.stop_level, st_stop + 4 * i, 4);
                std::memcpy(&j->result.interpreted_nodes, st_int + 8 * i, 8);
            } else {
                j->result.stop_level = -1;
                j->result.interpreted_nodes = (int64_t)j->ops.size();
                j->result.device_compiled = j->device_compiled ? 1 : 0;
                if (j->keep_resident) j->tree_in_pop = i;
            }
            j->result.status = GP_OK;
            j->t_done = t;
            j->result.latency_ms = t - j->t_submit;
            j->result.queue_ms = j->t_admit - j->t_submit;
            j->result.prep_ms = j->t_ready - j->t_submit;
            j->result.launch_ms = j->t_enq - j->t_admit;
            j->result.run_ms = t - j->t_enq;
            j->state = SJob::DONE;
            child_done(S, j);
        }
        S->slot_busy[b->slot] = 0;
        std::shared_ptr<ResidentBatch> rb;
        for (auto& j : b->jobs)
            if (b->kind == GP_JOB_FULL && j->keep_resident) {
                if (!rb) {
                    rb = std::make_shared<ResidentBatch>();
                    rb->pop = b->pop;
                    rb->bytes = b->bytes;
                }
                ++rb->refs;
                j->rb = rb;
                j->pop = rb->pop.get();
            }
        if (rb) b->bytes = 0;                     // charged to the resident batch instead
        b->pop.reset();
        b->parents.clear();
        S->graveyard.push_back(b);
        S->cv_disp.notify_all();
        S->cv_done.notify_all();
    }
}

}  // namespace
}  // namespace gpe

using namespace gpe;

extern "C" {

int gp_server_start(gp_ctx* ctxp, const gp_server_cfg* cfg)
{
    Ctx* ctx = (Ctx*)ctxp;
    if (!ctx) return GP_EINVAL;
    if (ctx->server) return set_err(ctx, GP_EINVAL, "server already running");
    (void)hipSetDevice(ctx->device);
    auto* S = new Server();
    S->ctx = ctx;
    S->cfg.n_streams = cfg && cfg->n_streams > 0 ? cfg->n_streams : 4;
    S->cfg.max_batch_jobs = cfg && cfg->max_batch_jobs > 0 ? cfg->max_batch_jobs : 64;
    S->cfg.prep_threads = cfg && cfg->prep_threads > 0 ? cfg->prep_threads : 8;
    S->cfg.budget_bytes = cfg ? cfg->budget_bytes : 0;
    S->cfg.device_compile_nodes = cfg ? cfg->device_compile_nodes : 0;
    S->device_compile_nodes = std::max<int64_t>(0, S->cfg.device_compile_nodes);
    S->budget = S->cfg.budget_bytes ? std::min<uint64_t>(S->cfg.budget_bytes, ctx->budget) : ctx->budget;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        S->tuned = ctx->tuned;
        S->forced_variant = ctx->forced_variant;
        S->forced_waves = ctx->forced_waves;
    }
    S->pinned_bytes = (size_t)S->cfg.max_batch_jobs * (20 + (size_t)16384 * 8);
    for (int i = 0; i < S->cfg.n_streams; ++i) {
        hipStream_t s = nullptr;
        void* h = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
            hipHostMalloc(&h, S->pinned_bytes, hipHostMallocDefault) != hipSuccess) {
            delete S;
            return set_err(ctx, GP_EDEVICE, "server stream or staging allocation failed");
        }
        S->streams.push_back(s);
        S->pinned.push_back(h);
    }
    for (int i = 0; i < S->cfg.prep_threads; ++i) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : S->streams) (void)hipStreamDestroy(x);
            for (auto x : S->prep_streams) (void)hipStreamDestroy(x);
            for (auto h : S->pinned) (void)hipHostFree(h);
            delete S;
            return set_err(ctx, GP_EDEVICE, "server stream allocation failed");
        }
        S->prep_streams.push_back(s);
        S->prep_arenas.push_back(std::make_unique<DevArena>());
    }
    S->slot_busy.assign(S->cfg.n_streams, 0);
    ctx->server = S;
    for (int i = 0; i < S->cfg.prep_threads; ++i) S->workers.emplace_back(prep_worker, S, i);
    S->dispatcher = std::thread(dispatch_loop, S);
    S->completer = std::thread(complete_loop, S);
    return GP_OK;
}

int gp_server_submit(gp_ctx* ctxp, const gp_job* job, int64_t* ticket)
{
    Ctx* ctx = (Ctx*)ctxp;
    if (!ctx || !job || !ticket) return GP_EINVAL;
    Server* S = ctx->server;
    if (!S) return set_err(ctx, GP_EINVAL, "server not started");
    if (job->kind != GP_JOB_FULL && job->kind != GP_JOB_INCREMENTAL) return set_err(ctx, GP_EINVAL, "unknown job kind");
    if (job->layout != GP_PREFIX && job->layout != GP_POSTFIX) return set_err(ctx, GP_EINVAL, "unknown layout");
    if (!job->ops || job->n_ops < 1) return set_err(ctx, GP_EINVAL, "empty tree");
    if (job->n_record_points < 0 || (job->n_record_points > 0 && !job->record_points))
        return set_err(ctx, GP_EINVAL, "bad record points");
    auto j = std::make_shared<SJob>();
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->cases.find(job->cases);
        if (it == ctx->cases.end()) return set_err(ctx, GP_EINVAL, "unknown case-set handle");
        j->cs = it->second;
    }
    j->kind = job->kind;
    j->layout = job->layout;
    j->cases_h = job->cases;
    j->ops.assign(job->ops, job->ops + job->n_ops);
    if (job->kind == GP_JOB_FULL) {
        j->points.assign(job->record_points, job->record_points + job->n_record_points);
        j->caller_points = j->points;
        for (int64_t q : j->points)
            if (q < 0 || q >= job->n_ops) return set_err(ctx, GP_EINVAL, "record point out of range");
        j->keep_resident = job->keep_resident != 0;
    } else {
        j->parent_ticket = job->parent_ticket;
        j->point = job->point;
    }
    // a lower bound of what the job needs on the device
    const uint64_t esz = j->cs->vtype == GP_BOOL ? 8 : 4;
    const uint64_t lower = (uint64_t)job->n_ops * 2 + (uint64_t)j->cs->stride * esz;
    std::lock_guard<std::mutex> lk(S->mu);
    if (lower > S->budget) return set_err(ctx, GP_EBUDGET, "job exceeds the server's HBM budget");
    if (job->kind == GP_JOB_INCREMENTAL) {
        auto pit = S->jobs.find(job->parent_ticket);
        if (pit == S->jobs.end() || pit->second->kind != GP_JOB_FULL || !pit->second->keep_resident)
            return set_err(ctx, GP_EINVAL, "parent ticket is not a resident full job");
        if (pit->second->cases_h != job->cases) return set_err(ctx, GP_EINVAL, "child and parent use different case sets");
        if (job->point < 0) return set_err(ctx, GP_EINVAL, "crossover point out of range");
        if (std::find(pit->second->caller_points.begin(), pit->second->caller_points.end(), job->point) ==
            pit->second->caller_points.end())
            return set_err(ctx, GP_ENOTFOUND, "point was not among the parent's record points");
    }
    if (job->kind == GP_JOB_INCREMENTAL) ++S->jobs.at(job->parent_ticket)->pending_children;
    j->ticket = S->next_ticket++;
    j->t_submit = now_ms();
    S->jobs[j->ticket] = j;
    S->arrived.push_back(j);
    *ticket = j->ticket;
    S->cv_prep.notify_one();
    return GP_OK;
}

int gp_server_poll(gp_ctx* ctxp, int64_t ticket, gp_job_result* out, void* root_out, int64_t root_cap)
{
    Ctx* ctx = (Ctx*)ctxp;
    if (!ctx || !out) return GP_EINVAL;
    Server* S = ctx->server;
    if (!S) return set_err(ctx, GP_EINVAL, "server not started");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return set_err(ctx, GP_EINVAL, "unknown ticket");
    SJob* j = it->second.get();
    if (j->state != SJob::DONE) return GP_EBUSY;
    if (root_out && (int64_t)j->root.size() > root_cap)
        return set_err(ctx, GP_EINVAL, "root_out holds " + std::to_string(root_cap) + " bytes; the job's output vector has " +
                                           std::to_string(j->root.size()));
    *out = j->result;
    out->root_bytes = (int64_t)j->root.size();
    if (root_out && !j->root.empty()) std::memcpy(root_out, j->root.data(), j->root.size());
    // results of jobs that are not resident parents are handed out once
    if (!(j->kind == GP_JOB_FULL && j->keep_resident)) S->jobs.erase(it);
    return GP_OK;
}

int gp_server_release(gp_ctx* ctxp, int64_t ticket)
{
    Ctx* ctx = (Ctx*)ctxp;
    if (!ctx) return GP_EINVAL;
    Server* S = ctx->server;
    if (!S) return set_err(ctx, GP_EINVAL, "server not started");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end() || it->second->kind != GP_JOB_FULL || !it->second->keep_resident)
        return set_err(ctx, GP_EINVAL, "ticket is not a resident full job");
    if (it->second->state != SJob::DONE) return GP_EBUSY;
    // children submitted and not done yet (arrived, being compiled, ready or
    // running) keep their parent
    if (it->second->pending_children > 0) return GP_EBUSY;
    std::shared_ptr<ResidentBatch> rb = it->second->rb;
    S->jobs.erase(it);
    if (rb && --rb->refs == 0) {
        // last resident parent of its batch: its memory goes back once freed
        auto b = std::make_shared<SBatch>();
        b->pop = rb->pop;
        b->bytes = rb->bytes;
        rb->pop.reset();
        S->graveyard.push_back(b);
    }
    S->cv_disp.notify_all();
    return GP_OK;
}

int gp_server_stop(gp_ctx* ctxp)
{
    Ctx* ctx = (Ctx*)ctxp;
    if (!ctx || !ctx->server) return GP_OK;
    Server* S = ctx->server;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        // let in-flight batches finish
        S->cv_done.notify_all();
        while (!S->inflight.empty()) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::milliseconds(1));
            lk.lock();
        }
        S->stopping = true;
    }
    S->cv_prep.notify_all();
    S->cv_disp.notify_all();
    S->cv_done.notify_all();
    for (auto& t : S->workers) t.join();
    S->dispatcher.join();
    S->completer.join();
    (void)hipSetDevice(ctx->device);
    for (auto s : S->streams) (void)hipStreamSynchronize(s);
    S->graveyard.clear();
    S->jobs.clear();
    S->ready.clear();
    S->arrived.clear();
    for (auto s : S->streams) (void)hipStreamDestroy(s);
    for (auto s : S->prep_streams) (void)hipStreamDestroy(s);
    S->prep_arenas.clear();
    for (auto h : S->pinned) (void)hipHostFree(h);
    ctx->server = nullptr;
    delete S;
    return GP_OK;
}

}  // extern "C"
