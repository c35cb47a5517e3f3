// Serving runtime: a request queue in front of several frames in flight.
//
// Each slot owns a renderer context (its own workspace), a HIP stream and a
// completion event, so frames of different requests run concurrently on the
// GPU and a new request starts as soon as any slot frees (continuous
// batching).  A request is admitted in arrival order when a slot is free and
// the workspace it needs fits the memory budget; idle slots give their
// workspace back when the head of the queue needs the room.  With graphs on,
// each (scene, image size, mode, statistics flag) is captured once per slot
// into a HIP graph; later requests copy their camera, options and output
// pointers into the slot's device frame record and replay the graph.  A
// frame that overflows its key capacity is re-queued at the front after the
// slot grows to the count the device reported.
#include <math.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "ctx.h"

using namespace dgs;

namespace {

constexpr int kMaxSlots = 16;
constexpr int kMaxAttempts = 4;

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct ShapeKey {
    int32_t scene, width, height, mode, stats;
    bool operator<(const ShapeKey& o) const {
        return std::tie(scene, width, height, mode, stats) < std::tie(o.scene, o.width, o.height, o.mode, o.stats);
    }
};

struct Request {
    int64_t id = 0;
    int32_t scene = 0;
    dgs_camera cam;
    dgs_render_opts opts;
    dgs_image out;
    FrameK frame;
    int mode = 0;
    ShapeKey shape;
    dgs_request_info info;
};

// Device side of the server.  Only the scheduler thread calls it.
class Executor {
public:
    virtual ~Executor() = default;
    virtual int num_slots() const = 0;
    virtual WorkspaceCaps caps(int slot) const = 0;
    // True when the slot holds a valid captured frame for this shape.
    virtual bool has_graph(int slot, const ShapeKey& k) const = 0;
    // Starts the frame (asynchronously); *graph = 1 replayed, 2 captured, 0 none.
    virtual dgs_status launch(int slot, const dgs_scene& s, Request& r, const WorkspaceCaps& want, int* graph,
                              std::string& err) = 0;
    // True once the slot's last frame has finished (or failed).
    virtual bool done(int slot) = 0;
    // Result of the finished frame; *keys receives the key count it produced.
    virtual dgs_status finish(int slot, int64_t* keys, std::string& err) = 0;
    virtual void release(int slot) = 0;
    virtual void shutdown() {}
};

// ------------------------------------------------------------------ HIP device

class DeviceExecutor final : public Executor {
    struct Slot {
        dgs_ctx ctx = nullptr;
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        FrameK* hframe = nullptr;   // pinned host copy source of the frame record
        uint32_t* hinfo = nullptr;  // pinned: [0] device error bits, [1] key count
        struct Graph {
            uint64_t generation;
            hipGraphExec_t exec;
        };
        std::map<ShapeKey, Graph> graphs;
    };
    int device_;
    bool graphs_;
    std::vector<Slot> slots_;

    void drop_graphs(Slot& s) {
        for (auto& g : s.graphs) hipGraphExecDestroy(g.second.exec);
        s.graphs.clear();
    }

public:
    DeviceExecutor(int device, int n, bool graphs) : device_(device), graphs_(graphs), slots_(n) {}

    dgs_status init(std::string& err) {
        hipSetDevice(device_);
        for (auto& s : slots_) {
            if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
                hipHostMalloc((void**)&s.hframe, sizeof(FrameK), hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void**)&s.hinfo, 2 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
                err = "stream, event or pinned buffer creation failed";
                return DGS_ERR_DEVICE;
            }
            s.hinfo[0] = s.hinfo[1] = 0;
            dgs_status st = dgs_create(device_, s.stream, &s.ctx);
            if (st == DGS_OK) s.ctx->two_streams = false;  // the slots overlap whole frames
            if (st != DGS_OK) {
                err = "context creation failed";
                return st;
            }
        }
        return DGS_OK;
    }

    ~DeviceExecutor() override { shutdown(); }

    void shutdown() override {
        hipSetDevice(device_);
        for (auto& s : slots_) {
            if (s.stream) hipStreamSynchronize(s.stream);
            drop_graphs(s);
            if (s.ctx) dgs_destroy(s.ctx);
            if (s.done) hipEventDestroy(s.done);
            if (s.stream) hipStreamDestroy(s.stream);
            if (s.hframe) hipHostFree(s.hframe);
            if (s.hinfo) hipHostFree(s.hinfo);
            s = Slot();
        }
    }

    int num_slots() const override { return (int)slots_.size(); }
    WorkspaceCaps caps(int slot) const override { return dgs_internal_caps(slots_[slot].ctx); }
    bool has_graph(int slot, const ShapeKey& k) const override {
        auto it = slots_[slot].graphs.find(k);
        return it != slots_[slot].graphs.end() && it->second.generation == slots_[slot].ctx->generation;
    }

    dgs_status launch(int slot, const dgs_scene& sc, Request& r, const WorkspaceCaps& want, int* graph,
                      std::string& err) override {
        Slot& s = slots_[slot];
        hipSetDevice(device_);
        *graph = 0;
        dgs_status st = dgs_internal_prepare(s.ctx, &sc, r.mode, r.cam.width, r.cam.height, want.keys);
        if (st != DGS_OK) {
            err = dgs_last_error(s.ctx);
            return st;
        }
        if (graphs_) {
            auto it = s.graphs.find(r.shape);
            if (it != s.graphs.end() && it->second.generation != s.ctx->generation) {
                hipGraphExecDestroy(it->second.exec);
                s.graphs.erase(it);
                it = s.graphs.end();
            }
            if (it == s.graphs.end()) {
                hipGraph_t g = nullptr;
                if (hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                    err = "graph capture could not start";
                    return DGS_ERR_DEVICE;
                }
                st = dgs_internal_render(s.ctx, &sc, &r.cam, &r.opts, &r.out, false);
                hipError_t e = hipStreamEndCapture(s.stream, &g);
                if (st != DGS_OK || e != hipSuccess) {
                    if (g) hipGraphDestroy(g);
                    err = st != DGS_OK ? dgs_last_error(s.ctx) : "graph capture failed";
                    return st != DGS_OK ? st : DGS_ERR_DEVICE;
                }
                hipGraphExec_t ex = nullptr;
                e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                hipGraphDestroy(g);
                if (e != hipSuccess) {
                    err = "graph instantiation failed";
                    return DGS_ERR_DEVICE;
                }
                it = s.graphs.emplace(r.shape, Slot::Graph{s.ctx->generation, ex}).first;
                *graph = 2;
            } else {
                *graph = 1;
            }
            *s.hframe = r.frame;  // the slot's previous frame has finished reading it
            if (hipMemcpyAsync(s.ctx->frame, s.hframe, sizeof(FrameK), hipMemcpyHostToDevice, s.stream) !=
                    hipSuccess ||
                hipGraphLaunch(it->second.exec, s.stream) != hipSuccess) {
                err = "graph launch failed";
                return DGS_ERR_DEVICE;
            }
        } else {
            st = dgs_internal_render(s.ctx, &sc, &r.cam, &r.opts, &r.out, true);
            if (st != DGS_OK) {
                err = dgs_last_error(s.ctx);
                return st;
            }
        }
        if (hipMemcpyAsync(s.hinfo, s.ctx->dev_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
            hipMemcpyAsync(s.hinfo + 1, s.ctx->misc, sizeof(uint32_t), hipMemcpyDeviceToHost, s.stream) !=
                hipSuccess ||
            hipEventRecord(s.done, s.stream) != hipSuccess) {
            err = "completion record failed";
            return DGS_ERR_DEVICE;
        }
        return DGS_OK;
    }

    bool done(int slot) override {
        hipError_t e = hipEventQuery(slots_[slot].done);
        return e != hipErrorNotReady;
    }

    dgs_status finish(int slot, int64_t* keys, std::string& err) override {
        Slot& s = slots_[slot];
        if (hipEventSynchronize(s.done) != hipSuccess) {
            err = "frame failed on the device";
            return DGS_ERR_DEVICE;
        }
        const uint32_t bits = s.hinfo[0];
        *keys = s.hinfo[1];
        if (bits) {
            hipMemsetAsync(s.ctx->dev_err, 0, sizeof(int), s.stream);
            hipStreamSynchronize(s.stream);
            if (bits & (1u << kErrTimeout)) {
                err = timeout_message((int)bits);
                return DGS_ERR_TIMEOUT;
            }
            if (bits & (1u << kErrCapacity)) {
                err = "key capacity exceeded";
                return DGS_ERR_CAPACITY;
            }
            err = "device error flag set";
            return DGS_ERR_DEVICE;
        }
        return DGS_OK;
    }

    void release(int slot) override {
        Slot& s = slots_[slot];
        drop_graphs(s);
        dgs_internal_release(s.ctx);
    }
};

// ------------------------------------------------------- simulated device

// Host-only stand-in with the same workspace accounting: a frame takes
// seconds_fixed + seconds_per_mpixel * W*H/1e6 and produces
// keys_per_pixel * W*H keys; more keys than the slot's capacity is reported
// as a capacity overflow, exactly as the device reports it.
class SimExecutor final : public Executor {
    struct Slot {
        WorkspaceCaps caps{0, 0, 0, 0};
        double busy_until = 0;
        int64_t keys = 0;
        bool overflow = false;
        std::map<ShapeKey, int> graphs;
    };
    dgs_sim_device sim_;
    bool graphs_;
    std::vector<Slot> slots_;

public:
    SimExecutor(const dgs_sim_device& sim, int n, bool graphs) : sim_(sim), graphs_(graphs), slots_(n) {}
    int num_slots() const override { return (int)slots_.size(); }
    WorkspaceCaps caps(int slot) const override { return slots_[slot].caps; }
    bool has_graph(int slot, const ShapeKey& k) const override { return slots_[slot].graphs.count(k) != 0; }

    dgs_status launch(int slot, const dgs_scene&, Request& r, const WorkspaceCaps& want, int* graph,
                      std::string&) override {
        Slot& s = slots_[slot];
        WorkspaceCaps nc = dgs_internal_plan(s.caps, want);
        if (memcmp(&nc, &s.caps, sizeof(nc)) != 0) s.graphs.clear();
        s.caps = nc;
        *graph = 0;
        if (graphs_) *graph = s.graphs.count(r.shape) ? 1 : 2;
        if (graphs_) s.graphs[r.shape] = 1;
        const double px = (double)r.cam.width * r.cam.height;
        s.keys = (int64_t)ceil(sim_.keys_per_pixel * px);
        s.overflow = s.keys > s.caps.keys;
        s.busy_until = now_s() + sim_.seconds_fixed + sim_.seconds_per_mpixel * px * 1e-6;
        return DGS_OK;
    }
    bool done(int slot) override { return now_s() >= slots_[slot].busy_until; }
    dgs_status finish(int slot, int64_t* keys, std::string& err) override {
        *keys = slots_[slot].keys;
        if (slots_[slot].overflow) {
            err = "key capacity exceeded";
            return DGS_ERR_CAPACITY;
        }
        return DGS_OK;
    }
    void release(int slot) override {
        slots_[slot].caps = WorkspaceCaps{0, 0, 0, 0};
        slots_[slot].graphs.clear();
    }
};

}  // namespace

// ------------------------------------------------------------------ server

struct dgs_server_s {
    std::unique_ptr<Executor> ex;
    dgs_server_config cfg;
    std::vector<dgs_scene> scenes;
    std::vector<bool> scene_has_cells;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<int64_t> queue;
    std::unordered_map<int64_t, Request> reqs;
    std::vector<int64_t> slot_req;  // request running in each slot, 0 = idle
    std::map<ShapeKey, int64_t> key_est;
    int64_t next_id = 1;
    bool stop = false;
    std::string err;
    dgs_server_stats st;
    std::thread th;

    int64_t held_bytes() const {
        int64_t b = 0;
        for (int s = 0; s < ex->num_slots(); s++) b += dgs_internal_bytes(ex->caps(s));
        return b;
    }

    WorkspaceCaps want_of(const Request& r) const {
        const dgs_scene& sc = scenes[r.scene];
        const int64_t M = sc.cell_offsets ? (int64_t)sc.num_gaussians : (int64_t)sc.num_cells * sc.gaussians_per_cell;
        const int64_t P = r.mode != DGS_MODE_ALPHA ? sc.num_cells : M;
        const int64_t tiles = (int64_t)((r.cam.width + kTile - 1) / kTile) * ((r.cam.height + kTile - 1) / kTile);
        auto it = key_est.find(r.shape);
        int64_t keys = it == key_est.end() ? dgs_internal_default_keys(P) : it->second + it->second / 4 + 4096;
        // no frame has more keys than (primitive, tile) pairs
        if (keys > P * tiles) keys = P * tiles > 1 ? P * tiles : 1;
        if (keys > (int64_t)(1u << 30)) keys = (int64_t)(1u << 30);
        return WorkspaceCaps{P, M, keys, tiles};
    }

    void finish_request(Request& r, int32_t state, dgs_status res) {
        r.info.state = state;
        r.info.result = res;
        r.info.t_done = now_s();
        if (state == DGS_REQ_DONE) st.completed++;
        if (state == DGS_REQ_FAILED) st.failed++;
        if (state == DGS_REQ_CANCELLED) st.cancelled++;
        cv_done.notify_all();
    }

    // Picks the next admissible (request, slot) in arrival order; frees idle
    // workspace when the head needs room; rejects requests that can never
    // fit.  Called with mu held.  Returns false when nothing can start.
    bool admit(int64_t* rid, int* slot, WorkspaceCaps* want) {
        while (!queue.empty()) {
            const int n = ex->num_slots();
            Request& r = reqs[queue.front()];
            const WorkspaceCaps w = want_of(r);
            int best = -1;
            int64_t best_delta = 0;
            bool best_graph = false;
            for (int s = 0; s < n; s++) {
                if (slot_req[s]) continue;
                const WorkspaceCaps c = ex->caps(s);
                const int64_t delta = dgs_internal_bytes(dgs_internal_plan(c, w)) - dgs_internal_bytes(c);
                // prefer no growth, then a slot that can replay this shape
                const bool replay = delta == 0 && ex->has_graph(s, r.shape);
                if (best < 0 || delta < best_delta || (delta == best_delta && replay && !best_graph)) {
                    best = s;
                    best_delta = delta;
                    best_graph = replay;
                }
            }
            if (best < 0) return false;  // every slot busy
            const int64_t alone = dgs_internal_bytes(dgs_internal_plan(WorkspaceCaps{0, 0, 0, 0}, w));
            if (cfg.memory_budget > 0 && alone > cfg.memory_budget) {
                queue.pop_front();
                r.info.result = DGS_ERR_OOM;
                err = "request needs more workspace than the memory budget";
                finish_request(r, DGS_REQ_FAILED, DGS_ERR_OOM);
                continue;
            }
            int64_t held = held_bytes();
            if (cfg.memory_budget > 0 && held + best_delta > cfg.memory_budget) {
                // give back the workspace of other idle slots, largest first
                for (;;) {
                    int victim = -1;
                    int64_t vb = 0;
                    for (int s = 0; s < n; s++) {
                        if (slot_req[s] || s == best) continue;
                        const int64_t b = dgs_internal_bytes(ex->caps(s));
                        if (b > vb) {
                            vb = b;
                            victim = s;
                        }
                    }
                    if (victim < 0 || held + best_delta <= cfg.memory_budget) break;
                    ex->release(victim);
                    st.releases++;
                    held -= vb;
                }
                if (held + best_delta > cfg.memory_budget) {
                    // the chosen slot's own workspace may be the one to drop
                    const int64_t own = dgs_internal_bytes(ex->caps(best));
                    if (held - own + alone <= cfg.memory_budget && own > 0) {
                        ex->release(best);
                        st.releases++;
                    } else {
                        return false;  // wait for running frames to finish
                    }
                }
            }
            queue.pop_front();
            *rid = r.id;
            *slot = best;
            *want = w;
            return true;
        }
        return false;
    }

    void loop() {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            bool progress = false;
            bool busy = false;
            // completions
            for (int s = 0; s < ex->num_slots(); s++) {
                if (!slot_req[s]) continue;
                if (!ex->done(s)) {
                    busy = true;
                    continue;
                }
                Request& r = reqs[slot_req[s]];
                slot_req[s] = 0;
                int64_t keys = 0;
                std::string e;
                dgs_status res = ex->finish(s, &keys, e);
                r.info.num_keys = keys;
                progress = true;
                if (res == DGS_ERR_CAPACITY && r.info.attempts < kMaxAttempts) {
                    // grow to what the frame produced and run it again first
                    int64_t& est = key_est[r.shape];
                    if (keys > est) est = keys;
                    st.retries++;
                    r.info.state = DGS_REQ_QUEUED;
                    queue.push_front(r.id);
                    continue;
                }
                if (res == DGS_OK) {
                    int64_t& est = key_est[r.shape];
                    if (keys > est) est = keys;
                    finish_request(r, DGS_REQ_DONE, DGS_OK);
                } else {
                    err = e;
                    finish_request(r, DGS_REQ_FAILED, res);
                }
            }
            // admissions
            int64_t rid;
            int slot;
            WorkspaceCaps want;
            while (admit(&rid, &slot, &want)) {
                Request& r = reqs[rid];
                r.info.state = DGS_REQ_RUNNING;
                r.info.slot = slot;
                r.info.attempts++;
                if (r.info.attempts == 1) r.info.t_start = now_s();
                slot_req[slot] = rid;
                int graph = 0;
                std::string e;
                const dgs_scene sc = scenes[r.scene];
                lk.unlock();
                dgs_status res = ex->launch(slot, sc, r, want, &graph, e);
                lk.lock();
                progress = true;
                if (graph == 1) st.graph_replays++;
                if (graph == 2) st.graph_captures++;
                r.info.graph = graph;
                if (res != DGS_OK) {
                    slot_req[slot] = 0;
                    err = e;
                    finish_request(r, DGS_REQ_FAILED, res);
                    continue;
                }
                busy = true;
                const int64_t b = held_bytes();
                if (b > st.peak_workspace_bytes) st.peak_workspace_bytes = b;
            }
            if (stop && !busy) {
                for (int64_t id : queue) finish_request(reqs[id], DGS_REQ_CANCELLED, DGS_OK);
                queue.clear();
                break;
            }
            if (progress) continue;
            if (busy) {
                // frames in flight: poll their events without holding the lock long
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            } else {
                cv_work.wait_for(lk, std::chrono::milliseconds(5));
            }
        }
    }
};

namespace {

dgs_status server_start(dgs_server srv, dgs_server* out) {
    srv->slot_req.assign(srv->ex->num_slots(), 0);
    memset(&srv->st, 0, sizeof(srv->st));
    srv->th = std::thread([srv] { srv->loop(); });
    *out = srv;
    return DGS_OK;
}

dgs_status check_config(const dgs_server_config* cfg) {
    if (!cfg || cfg->num_slots < 1 || cfg->num_slots > kMaxSlots || cfg->memory_budget < 0)
        return DGS_ERR_INVALID_ARG;
    return DGS_OK;
}

}  // namespace

extern "C" {

void dgs_server_default_config(dgs_server_config* cfg) {
    if (!cfg) return;
    cfg->num_slots = 4;
    cfg->use_graphs = 1;
    cfg->memory_budget = 0;
}

dgs_status dgs_server_create(int device, const dgs_server_config* cfg, dgs_server* out) {
    if (!out || check_config(cfg) != DGS_OK) return DGS_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DGS_ERR_INVALID_ARG;
    auto* ex = new DeviceExecutor(device, cfg->num_slots, cfg->use_graphs != 0);
    std::string e;
    dgs_status st = ex->init(e);
    if (st != DGS_OK) {
        delete ex;
        return st;
    }
    dgs_server srv = new dgs_server_s();
    srv->ex.reset(ex);
    srv->cfg = *cfg;
    return server_start(srv, out);
}

dgs_status dgs_server_create_simulated(const dgs_server_config* cfg, const dgs_sim_device* sim, dgs_server* out) {
    if (!out || !sim || check_config(cfg) != DGS_OK) return DGS_ERR_INVALID_ARG;
    if (!(sim->seconds_fixed >= 0) || !(sim->seconds_per_mpixel >= 0) || !(sim->keys_per_pixel >= 0))
        return DGS_ERR_INVALID_ARG;
    *out = nullptr;
    dgs_server srv = new dgs_server_s();
    srv->ex.reset(new SimExecutor(*sim, cfg->num_slots, cfg->use_graphs != 0));
    srv->cfg = *cfg;
    return server_start(srv, out);
}

dgs_status dgs_server_add_scene(dgs_server srv, const dgs_scene* scene, int32_t* scene_id) {
    if (!srv || !scene || !scene_id) return DGS_ERR_INVALID_ARG;
    dgs_ctx_s tmp;
    dgs_status st = dgs_internal_check_scene(&tmp, scene, DGS_MODE_ALPHA);
    std::lock_guard<std::mutex> lk(srv->mu);
    if (st != DGS_OK) {
        srv->err = tmp.err;
        return st;
    }
    srv->scenes.push_back(*scene);
    srv->scene_has_cells.push_back(dgs_internal_check_scene(&tmp, scene, DGS_MODE_DUPLEX) == DGS_OK);
    *scene_id = (int32_t)srv->scenes.size() - 1;
    return DGS_OK;
}

dgs_status dgs_server_submit(dgs_server srv, int32_t scene_id, const dgs_camera* cam, const dgs_render_opts* opts,
                             const dgs_image* out, int64_t* request_id) {
    if (!srv || !request_id) return DGS_ERR_INVALID_ARG;
    Request r;
    dgs_ctx_s tmp;
    dgs_status st = dgs_internal_frame(&tmp, cam, opts, out, &r.frame, &r.mode);
    std::lock_guard<std::mutex> lk(srv->mu);
    if (st != DGS_OK) {
        srv->err = tmp.err;
        return st;
    }
    if (srv->stop) {
        srv->err = "server is shutting down";
        return DGS_ERR_INVALID_ARG;
    }
    if (scene_id < 0 || scene_id >= (int32_t)srv->scenes.size()) {
        srv->err = "unknown scene id";
        return DGS_ERR_INVALID_ARG;
    }
    if (r.mode != DGS_MODE_ALPHA && !srv->scene_has_cells[scene_id]) {
        srv->err = "a Duplex or LC-WSR render needs the scene's cell arrays";
        return DGS_ERR_INVALID_ARG;
    }
    r.id = srv->next_id++;
    r.scene = scene_id;
    r.cam = *cam;
    dgs_default_opts(&r.opts);
    if (opts) r.opts = *opts;
    r.out = *out;
    r.shape = ShapeKey{scene_id, cam->width, cam->height, r.mode, (int32_t)r.frame.o.stats};
    memset(&r.info, 0, sizeof(r.info));
    r.info.state = DGS_REQ_QUEUED;
    r.info.slot = -1;
    r.info.t_submit = now_s();
    *request_id = r.id;
    srv->reqs.emplace(r.id, r);
    srv->queue.push_back(r.id);
    srv->st.submitted++;
    srv->cv_work.notify_one();
    return DGS_OK;
}

dgs_status dgs_server_query(dgs_server srv, int64_t request_id, dgs_request_info* info) {
    if (!srv || !info) return DGS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(request_id);
    if (it == srv->reqs.end()) return DGS_ERR_INVALID_ARG;
    *info = it->second.info;
    return DGS_OK;
}

dgs_status dgs_server_wait(dgs_server srv, int64_t request_id, double timeout_s, dgs_request_info* info) {
    if (!srv) return DGS_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto finished = [&] {
        auto it = srv->reqs.find(request_id);
        return it == srv->reqs.end() || it->second.info.state >= DGS_REQ_DONE;
    };
    if (timeout_s < 0) {
        srv->cv_done.wait(lk, finished);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), finished)) {
        return DGS_ERR_TIMEOUT;
    }
    auto it = srv->reqs.find(request_id);
    if (it == srv->reqs.end()) return DGS_ERR_INVALID_ARG;
    if (info) *info = it->second.info;
    return DGS_OK;
}

dgs_status dgs_server_cancel(dgs_server srv, int64_t request_id) {
    if (!srv) return DGS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(request_id);
    if (it == srv->reqs.end() || it->second.info.state != DGS_REQ_QUEUED) return DGS_ERR_INVALID_ARG;
    for (auto q = srv->queue.begin(); q != srv->queue.end(); ++q)
        if (*q == request_id) {
            srv->queue.erase(q);
            break;
        }
    srv->finish_request(it->second, DGS_REQ_CANCELLED, DGS_OK);
    return DGS_OK;
}

dgs_status dgs_server_release(dgs_server srv, int64_t request_id) {
    if (!srv) return DGS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(request_id);
    if (it == srv->reqs.end() || it->second.info.state < DGS_REQ_DONE) return DGS_ERR_INVALID_ARG;
    srv->reqs.erase(it);
    return DGS_OK;
}

dgs_status dgs_server_get_stats(dgs_server srv, dgs_server_stats* out) {
    if (!srv || !out) return DGS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->st;
    out->workspace_bytes = srv->held_bytes();
    out->queued = (int64_t)srv->queue.size();
    int64_t running = 0;
    for (int64_t r : srv->slot_req) running += r != 0;
    out->running = running;
    return DGS_OK;
}

const char* dgs_server_last_error(dgs_server srv) {
    if (!srv) return "NULL server";
    std::lock_guard<std::mutex> lk(srv->mu);
    thread_local std::string copy;
    copy = srv->err;
    return copy.c_str();
}

dgs_status dgs_server_destroy(dgs_server srv) {
    if (!srv) return DGS_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        for (int64_t id : srv->queue) srv->finish_request(srv->reqs[id], DGS_REQ_CANCELLED, DGS_OK);
        srv->queue.clear();
        srv->cv_work.notify_one();
    }
    srv->th.join();
    srv->ex->shutdown();
    delete srv;
    return DGS_OK;
}

}  // extern "C"
